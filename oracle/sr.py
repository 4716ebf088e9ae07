"""Oracle for the stochastic-reconfiguration step (test infrastructure).

TEST INFRASTRUCTURE ONLY: the correctness reference for the GPU library's
SR calls.  Only the tests and the benchmark's CPU-baseline leg may import
it; the library and its Python binding never do.

What it computes, in plain numpy FP64, following the paper's section
"ANQS-tailored stochastic reconfiguration":

  - the SR sample set: the N_SR unique samples of highest probability
    p(x) = |psi(x)|^2 (largest Re log psi), ties to the lower sample index;
  - their renormalised probabilities w_x = p(x) / sum_{y in set} p(y) (the
    renormalised probabilities of Eq. variational_energy, restricted to the
    set), instead of occurrence numbers;
  - the quantum geometric tensor of Eq. qgt_definition estimated over that
    set, S_pq = sum_x w_x conj(O_xp - Obar_p) (O_xq - Obar_q) with
    O_xp = d log psi(x) / d theta_p and Obar_p = sum_x w_x O_xp; the
    parameters are real, so the real part Re S is the metric;
  - the SR-transformed gradient: the solution of (Re S + lambda I) d = F for
    a given energy gradient F (Eq. grad_def), lambda > 0 a diagonal shift.

Each function is the plain definition: S is formed as an N_p x N_p matrix
and the system is solved directly (numpy.linalg.solve), which is only
feasible for small N_p.
"""
from __future__ import annotations

import numpy as np


def select(logpsi: np.ndarray, n_sr: int) -> np.ndarray:
    """Indices of the n_sr samples with the largest Re log psi, in that
    order (descending), ties broken by the lower index."""
    re = np.asarray(logpsi).real
    order = sorted(range(re.size), key=lambda i: (-re[i], i))
    return np.array(order[:n_sr], dtype=np.int64)


def weights(logpsi_set: np.ndarray) -> np.ndarray:
    """Renormalised probabilities |psi|^2 / sum |psi|^2 over the set."""
    re = np.asarray(logpsi_set).real
    p = np.exp(2.0 * (re - re.max()))
    return p / p.sum()


def qgt(O: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Complex S_pq = sum_x w_x conj(O_xp - Obar_p)(O_xq - Obar_q)."""
    O = np.asarray(O, dtype=np.complex128)
    w = np.asarray(w, dtype=np.float64)
    obar = w @ O
    D = O - obar[None, :]
    return (D.conj().T * w[None, :]) @ D


def sr_solve(O: np.ndarray, w: np.ndarray, F: np.ndarray, lam: float) -> np.ndarray:
    """d = (Re S + lambda I)^{-1} F."""
    S = qgt(O, w).real
    return np.linalg.solve(S + lam * np.eye(S.shape[0]), np.asarray(F, dtype=np.float64))
