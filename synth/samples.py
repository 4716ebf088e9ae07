"""Seeded unique sample batches U, log-amplitudes and weights (inputs only).

A batch stands in for what the paper's autoregressive sampler without
replacement returns: N_unq distinct bit-packed basis vectors (Sec. "GPU
implementation", compressed storage) with complex log-amplitudes
log psi = log|psi| + i phi from the ansatz.  Recipe:

* the Hartree-Fock determinant (first n_e qubits occupied) is always in U;
* other samples are excitations of rank k in {1..4}, P(k) ~ 0.5^k: k distinct
  occupied spin orbitals chosen uniformly, each moved to a distinct virtual
  spin orbital of the same spin, chosen uniformly (particle number and S_z
  conserved);
* duplicates are rejected in draw order until |U| = N_unq, then U is shuffled
  so that keys arrive unsorted;
* log|psi| = -k + N(0, 0.3^2), phase ~ U(0, 2 pi), with k the excitation rank
  (ceil(popcount(x ^ x_HF) / 2) for states outside the sector).

Keys: uint64 array [N_unq, W], qubit q in word q // 64, bit q % 64.
"""
from __future__ import annotations

import itertools

import numpy as np

_ONE = np.uint64(1)


def n_words(n_qubits: int) -> int:
    return (n_qubits + 63) // 64


def key_from_bits(bits: np.ndarray) -> np.ndarray:
    """bits: [M, N] 0/1 -> keys [M, W]."""
    M, N = bits.shape
    W = n_words(N)
    keys = np.zeros((M, W), dtype=np.uint64)
    for q in range(N):
        keys[:, q // 64] |= bits[:, q].astype(np.uint64) << np.uint64(q % 64)
    return keys


def bits_from_key(keys: np.ndarray, n_qubits: int) -> np.ndarray:
    out = np.zeros((keys.shape[0], n_qubits), dtype=np.uint8)
    for q in range(n_qubits):
        out[:, q] = ((keys[:, q // 64] >> np.uint64(q % 64)) & _ONE).astype(np.uint8)
    return out


def hf_bits(n_qubits: int, n_electrons: int) -> np.ndarray:
    b = np.zeros(n_qubits, dtype=np.uint8)
    b[:n_electrons] = 1
    return b


def popcount_rows(keys: np.ndarray) -> np.ndarray:
    out = np.zeros(keys.shape[0], dtype=np.int64)
    for w in range(keys.shape[1]):
        v = keys[:, w].copy()
        for s in range(64):
            out += ((v >> np.uint64(s)) & _ONE).astype(np.int64)
    return out


def _rows_as_void(keys: np.ndarray) -> np.ndarray:
    k = np.ascontiguousarray(keys)
    return k.view(np.dtype((np.void, k.dtype.itemsize * k.shape[1]))).ravel()


def excitation_batch(n_qubits: int, n_electrons: int, n_unique: int,
                     rng: np.random.Generator, max_rank: int = 4) -> tuple[np.ndarray, np.ndarray]:
    """Return (keys [M, W] shuffled, rank [M])."""
    N, ne = n_qubits, n_electrons
    hf = hf_bits(N, ne)
    occ = np.arange(ne)
    vir = np.arange(ne, N)
    occ_s = [occ[occ % 2 == s] for s in (0, 1)]
    vir_s = [vir[vir % 2 == s] for s in (0, 1)]
    ranks = np.arange(1, max_rank + 1)
    pk = 0.5 ** ranks
    pk = pk / pk.sum()

    accepted_keys = [key_from_bits(hf[None, :])]
    accepted_rank = [np.zeros(1, dtype=np.int64)]
    seen = set(_rows_as_void(accepted_keys[0]).tolist())
    have = 1
    while have < n_unique:
        need = n_unique - have
        B = max(1024, 2 * need)
        k = rng.choice(ranks, size=B, p=pk)
        bits = np.repeat(hf[None, :], B, axis=0)
        # holes: first k of a random permutation of the occupied modes
        perm = np.argsort(rng.random((B, ne)), axis=1)
        hole = perm < k[:, None]                     # hole[b, position in occ]
        bits[:, :ne] ^= hole.astype(np.uint8)
        for s in (0, 1):
            ks = hole[:, occ_s[s]].sum(axis=1)       # holes of spin s
            nv = vir_s[s].size
            vperm = np.argsort(rng.random((B, nv)), axis=1)
            part = vperm < ks[:, None]
            cols = vir_s[s]
            bits[:, cols] ^= part.astype(np.uint8)
        keys = key_from_bits(bits)
        v = _rows_as_void(keys)
        _, first = np.unique(v, return_index=True)
        first.sort()
        take = []
        for i in first:
            kv = v[i].tobytes()
            if kv in seen:
                continue
            seen.add(kv)
            take.append(i)
            if len(take) == need:
                break
        take = np.array(take, dtype=np.int64)
        accepted_keys.append(keys[take])
        accepted_rank.append(k[take])
        have += take.size
    keys = np.concatenate(accepted_keys)
    rank = np.concatenate(accepted_rank)
    order = rng.permutation(keys.shape[0])
    return np.ascontiguousarray(keys[order]), rank[order]


def sector_plus_random(n_qubits: int, n_alpha: int, n_beta: int, n_unique: int,
                       rng: np.random.Generator) -> np.ndarray:
    """All determinants of the (n_alpha, n_beta) sector plus states drawn
    uniformly without replacement from the rest of the 2^N basis, shuffled.
    Used where the sector alone is smaller than the requested batch."""
    N = n_qubits
    assert N <= 24
    a_modes = list(range(0, N, 2))
    b_modes = list(range(1, N, 2))
    sector = []
    for ca in itertools.combinations(a_modes, n_alpha):
        for cb in itertools.combinations(b_modes, n_beta):
            sector.append(sum(1 << q for q in ca + cb))
    sector = np.array(sorted(sector), dtype=np.uint64)
    assert sector.size <= n_unique
    rest = np.setdiff1d(np.arange(2 ** N, dtype=np.uint64), sector)
    extra = rng.choice(rest, size=n_unique - sector.size, replace=False)
    keys = np.concatenate([sector, extra])[:, None]
    return np.ascontiguousarray(keys[rng.permutation(keys.shape[0])])


def excitation_rank(keys: np.ndarray, n_qubits: int, n_electrons: int) -> np.ndarray:
    hf = key_from_bits(hf_bits(n_qubits, n_electrons)[None, :])
    return (popcount_rows(keys ^ hf) + 1) // 2


def log_amplitudes(rank: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """complex128 [M]: log|psi| = -k + N(0, 0.3^2), phase ~ U(0, 2 pi)."""
    re = -rank.astype(np.float64) + rng.normal(0.0, 0.3, size=rank.size)
    im = rng.uniform(0.0, 2 * np.pi, size=rank.size)
    return re + 1j * im


def multinomial_counts(logpsi: np.ndarray, total: int, rng: np.random.Generator) -> np.ndarray:
    """w = 1 + Multinomial(total - M, p ~ |psi|^2): every sample counted once."""
    lp = 2.0 * logpsi.real
    p = np.exp(lp - lp.max())
    p /= p.sum()
    return 1.0 + rng.multinomial(total - logpsi.size, p).astype(np.float64)
