"""Pins of the SR oracle (oracle/sr.py) against facts fixed outside it: the
quantum geometric tensor of Eq. qgt_definition computed from finite
differences of a normalised state vector, its invariance under a constant
shift of log psi, a brute-force selection of the highest-probability samples,
and the limits of the shifted solve."""
import numpy as np
import pytest

from oracle import sr


def _model(theta, F, G):
    """log psi(x) = sum_p theta_p F_xp + 0.3 (sum_p theta_p G_xp)^2 over all
    basis states x (complex features), and its exact log-derivatives."""
    a = F @ theta
    b = G @ theta
    logpsi = a + 0.3 * b * b
    O = F + 0.6 * b[:, None] * G
    return logpsi, O


@pytest.mark.parametrize("seed", [0, 1])
def test_qgt_is_the_metric_of_the_normalised_state(seed):
    """With the whole basis as the sample set and w = |psi|^2 / sum |psi|^2,
    the estimator equals <d_p psi|d_q psi> - <d_p psi|psi><psi|d_q psi> of the
    normalised state, its derivatives taken by central finite differences."""
    rng = np.random.default_rng(seed)
    D, P = 8, 5
    F = rng.normal(size=(D, P)) + 1j * rng.normal(size=(D, P))
    G = 0.5 * (rng.normal(size=(D, P)) + 1j * rng.normal(size=(D, P)))
    theta = 0.3 * rng.normal(size=P)

    def state(t):
        lp, _ = _model(t, F, G)
        v = np.exp(lp)
        return v / np.linalg.norm(v)

    h = 1e-6
    psi = state(theta)
    dpsi = np.empty((P, D), dtype=complex)
    for p in range(P):
        e = np.zeros(P)
        e[p] = h
        dpsi[p] = (state(theta + e) - state(theta - e)) / (2 * h)
    S_fd = dpsi.conj() @ dpsi.T - np.outer(dpsi.conj() @ psi, psi.conj() @ dpsi.T)
    lp, O = _model(theta, F, G)
    S = sr.qgt(O, sr.weights(lp))
    np.testing.assert_allclose(S, S_fd, atol=1e-7)


def test_qgt_shift_invariance():
    """A constant added to every O_x (a parameter that only rescales psi)
    does not change S; neither does a constant added to log psi."""
    rng = np.random.default_rng(3)
    O = rng.normal(size=(30, 7)) + 1j * rng.normal(size=(30, 7))
    L = rng.normal(size=30) + 1j * rng.normal(size=30)
    S = sr.qgt(O, sr.weights(L))
    np.testing.assert_allclose(sr.qgt(O + (0.7 - 2.0j), sr.weights(L)), S, atol=1e-12)
    np.testing.assert_allclose(sr.qgt(O, sr.weights(L + 40.0)), S, atol=1e-12)
    assert np.allclose(S, S.conj().T) and np.linalg.eigvalsh(S).min() > -1e-12


def test_select_brute_force():
    rng = np.random.default_rng(4)
    re = rng.integers(-5, 5, size=300).astype(float)       # many ties
    L = re + 1j * rng.uniform(0, 6, 300)
    idx = sr.select(L, 40)
    want = np.lexsort((np.arange(300), -re))[:40]
    np.testing.assert_array_equal(idx, want)
    w = sr.weights(L[idx])
    assert abs(w.sum() - 1) < 1e-15
    np.testing.assert_allclose(w / w[0], np.exp(2 * (re[idx] - re[idx[0]])), rtol=1e-14)


def test_solve_limits():
    """Without curvature (all samples with the same log-derivatives) S = 0
    and d = F / lambda; for any O the residual of (Re S + lambda I) d = F
    vanishes and a large shift gives d -> F / lambda."""
    rng = np.random.default_rng(5)
    P = 12
    F = rng.normal(size=P)
    L = rng.normal(size=9) + 0j
    row = rng.normal(size=P) + 1j * rng.normal(size=P)
    d = sr.sr_solve(np.tile(row, (9, 1)), sr.weights(L), F, 0.25)
    np.testing.assert_allclose(d, F / 0.25, rtol=1e-13)
    O = rng.normal(size=(9, P)) + 1j * rng.normal(size=(9, P))
    d = sr.sr_solve(O, sr.weights(L), F, 1e-3)
    S = sr.qgt(O, sr.weights(L)).real
    np.testing.assert_allclose(S @ d + 1e-3 * d, F, atol=1e-9)
    d = sr.sr_solve(O, sr.weights(L), F, 1e9)
    np.testing.assert_allclose(d * 1e9, F, rtol=1e-6)
