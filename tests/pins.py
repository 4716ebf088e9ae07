"""Independent references used to pin the oracle and the input generator.

Nothing here uses the bit-mask phase rule of Eq. pauli_melem; each reference
comes from a different formulation of the same physics:

* dense_pauli      - Pauli strings as tensor products of the textbook 2x2
                     matrices (I, X, Y, Z), entry by entry;
* dense_fermion    - second-quantised H applied to occupation-number vectors
                     with the Jordan-Wigner sign (-1)^(occupied modes below);
* slater_condon    - closed-form diagonal energy of a determinant.
"""
from __future__ import annotations

import numpy as np

PAULI = {
    "I": np.eye(2, dtype=complex),
    "X": np.array([[0, 1], [1, 0]], dtype=complex),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=complex),
    "Z": np.array([[1, 0], [0, -1]], dtype=complex),
}


def letters(n_qubits, xy_row, yz_row):
    """Decode one term's masks into letters per qubit (X = XY&~YZ, Y = XY&YZ,
    Z = ~XY&YZ), following the definitions XY = X|Y and YZ = Y|Z."""
    out = []
    for q in range(n_qubits):
        w, b = divmod(q, 64)
        a = (int(xy_row[w]) >> b) & 1
        c = (int(yz_row[w]) >> b) & 1
        out.append({(0, 0): "I", (1, 0): "X", (1, 1): "Y", (0, 1): "Z"}[(a, c)])
    return out


def dense_pauli_kron(ham) -> np.ndarray:
    """sum_l h_l (P_{N-1} kron ... kron P_0); basis index = sum_q x_q 2^q."""
    N = ham.n_qubits
    H = np.zeros((2 ** N, 2 ** N), dtype=complex)
    for l in range(ham.n_terms):
        ls = letters(N, ham.xy[l], ham.yz[l])
        m = np.ones((1, 1), dtype=complex)
        for q in range(N):
            m = np.kron(PAULI[ls[q]], m)
        H += ham.coeff[l] * m
    return H


def dense_pauli(ham) -> np.ndarray:
    """Same matrix as dense_pauli_kron, built column by column: each tensor
    product of 2x2 matrices has one non-zero per column, the product over
    qubits of the single-qubit entries."""
    N = ham.n_qubits
    D = 2 ** N
    cols = np.arange(D)
    H = np.zeros((D, D), dtype=complex)
    for l in range(ham.n_terms):
        ls = letters(N, ham.xy[l], ham.yz[l])
        rows = np.zeros(D, dtype=np.int64)
        val = np.ones(D, dtype=complex)
        for q in range(N):
            m = PAULI[ls[q]]
            cb = (cols >> q) & 1
            nz = np.argmax(np.abs(m), axis=0)        # row with the non-zero, per column
            rb = nz[cb]
            val *= m[rb, cb]
            rows |= rb << q
        np.add.at(H, (rows, cols), ham.coeff[l] * val)
    return H


def _spin_orbital_tensors(h, g):
    n = h.shape[0]
    N = 2 * n
    sp = np.arange(N) // 2
    spin = np.arange(N) % 2
    t = np.where(spin[:, None] == spin[None, :], h[sp][:, sp], 0.0)
    same = spin[:, None] == spin[None, :]
    gso = g[np.ix_(sp, sp, sp, sp)] * same[:, :, None, None] * same[None, None, :, :]
    return t, gso


def _annihilate(states, mode):
    occ = (states >> mode) & 1
    sign = 1 - 2 * (np.array([bin(int(s) & ((1 << mode) - 1)).count("1") for s in states]) & 1)
    return np.where(occ == 1, states ^ (1 << mode), -1), np.where(occ == 1, sign, 0)


def _create(states, mode):
    occ = (states >> mode) & 1
    sign = 1 - 2 * (np.array([bin(int(s) & ((1 << mode) - 1)).count("1") for s in states]) & 1)
    ok = (occ == 0) & (states >= 0)
    return np.where(ok, states | (1 << mode), -1), np.where(ok, sign, 0)


def dense_fermion(h, g, basis=None) -> np.ndarray:
    """<y| H |x> for H = sum t_PQ a+_P a_Q + 1/2 sum g_PQRS a+_P a+_R a_S a_Q
    over the given basis (all 2^N occupation vectors by default)."""
    t, gso = _spin_orbital_tensors(h, g)
    N = t.shape[0]
    basis = np.arange(2 ** N) if basis is None else np.asarray(basis, dtype=np.int64)
    index = {int(b): i for i, b in enumerate(basis)}
    H = np.zeros((basis.size, basis.size))

    def add(final, amp):
        for col in np.flatnonzero(amp != 0):
            row = index.get(int(final[col]))
            if row is not None:
                H[row, col] += amp[col]

    for Pm in range(N):
        for Qm in range(N):
            if t[Pm, Qm] == 0:
                continue
            s1, f1 = _annihilate(basis, Qm)
            s1 = np.where(f1 != 0, s1, 0)
            s2, f2 = _create(s1, Pm)
            add(s2, t[Pm, Qm] * f1 * f2)
    nz = np.argwhere(gso != 0)
    for Pm, Qm, Rm, Sm in nz:
        s1, f1 = _annihilate(basis, Qm)
        s1 = np.where(f1 != 0, s1, 0)
        s2, f2 = _annihilate(s1, Sm)
        s2 = np.where(f2 != 0, s2, 0)
        s3, f3 = _create(s2, Rm)
        s3 = np.where(f3 != 0, s3, 0)
        s4, f4 = _create(s3, Pm)
        add(s4, 0.5 * gso[Pm, Qm, Rm, Sm] * f1 * f2 * f3 * f4)
    return H


def slater_condon(h, g, occupied) -> float:
    """E = sum_{P in occ} t_PP + 1/2 sum_{P,Q in occ} [(PP|QQ) - (PQ|QP)]."""
    t, gso = _spin_orbital_tensors(h, g)
    occ = np.asarray(list(occupied), dtype=np.int64)
    e = t[occ, occ].sum()
    two = 0.0
    for Pm in occ:
        for Qm in occ:
            two += gso[Pm, Pm, Qm, Qm] - gso[Pm, Qm, Qm, Pm]
    return float(e + 0.5 * two)


def occupied_modes(key_words, n_qubits):
    return [q for q in range(n_qubits) if (int(key_words[q // 64]) >> (q % 64)) & 1]
