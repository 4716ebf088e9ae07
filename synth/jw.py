"""Seeded synthetic Jordan-Wigner qubit Hamiltonians (input generation only).

The paper's molecular Hamiltonians (Sec. "Ab initio quantum chemistry", Eqs.
fermionic_qc and jw_hamiltonian) come from chemistry packages that are not
available here, so workloads are built from random integrals instead:

  H = sum_{pq,s} h_pq a+_{ps} a_{qs}
      + 1/2 sum_{pqrs,st} (pq|rs) a+_{ps} a+_{rt} a_{st} a_{qs}

over n spatial orbitals (chemist's notation, no nuclear repulsion).  Spin
orbital P = 2p + spin (alpha = 0), so the Hartree-Fock determinant occupies
the first n_e qubits as the paper states for x_HF.  Jordan-Wigner with |1> =
occupied: a_P = Z_0 ... Z_{P-1} (X_P + i Y_P)/2.

Output is the paper's term encoding (Sec. "Hamiltonian arithmetic"): real
coefficient h_l plus the bit vectors XY_l = X|Y and YZ_l = Y|Z, qubit q stored
in word q // 64, bit q % 64.  Nothing here evaluates matrix elements or local
energies; that is the method's arithmetic and lives elsewhere.

Construction: H is split by the set F of qubits a term flips (its XY mask):
  * F empty      - number operators n_P and n_A n_B, closed form;
  * |F| = 2      - one-body hopping plus the two-body terms n_R a+_P a_Q;
  * |F| = 4      - two-body double excitations, three pairings per 4-set.
For |F| > 0 each fermionic monomial is a product of Pauli operators on its own
k <= 4 qubits times a Z string on the qubits strictly between its indices
(Z_m appears iff an odd number of the monomial's indices exceed m).  The local
2^k x 2^k matrix of each monomial pattern is formed numerically from sigma
matrices and expanded in Pauli strings by traces, once per pattern; all index
tuples of that pattern are then placed with vectorised bit arithmetic.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

SEED_BASE = 240807625


def rng_for(cfg: int, stream: int) -> np.random.Generator:
    """Generator for (configuration id, stream id); streams: 0 integrals,
    1 samples, 2 log-amplitudes, 3 weights, 4 batch plan, 100+k problem k."""
    return np.random.default_rng([SEED_BASE, cfg, stream])


# ----------------------------------------------------------------------------
# integrals
# ----------------------------------------------------------------------------
def spatial_integrals(n: int, rng: np.random.Generator):
    """h_pq symmetric ~ N(0,1) exp(-|p-q|/4); (pq|rs) 8-fold symmetric
    ~ N(0, 0.5^2) exp(-(|p-q|+|r-s|)/4).  Values are drawn for canonical
    index sets in row-major order and mirrored."""
    h = np.zeros((n, n))
    p, q = np.triu_indices(n)
    vals = rng.normal(0.0, 1.0, size=p.size) * np.exp(-np.abs(p - q) / 4.0)
    h[p, q] = vals
    h[q, p] = vals

    a, b = np.tril_indices(n)            # compound index pq = a(a+1)/2 + b, a >= b
    npair = a.size
    i1, i2 = np.tril_indices(npair)      # pq >= rs
    p, q, r, s = a[i1], b[i1], a[i2], b[i2]
    vals = rng.normal(0.0, 0.5, size=p.size) * np.exp(-(np.abs(p - q) + np.abs(r - s)) / 4.0)
    g = np.zeros((n, n, n, n))
    for (w, x, y, z) in ((p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                         (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)):
        g[w, x, y, z] = vals
    return h, g


# ----------------------------------------------------------------------------
# local Pauli expansion of fermionic monomials
# ----------------------------------------------------------------------------
_PAULI = {
    "I": np.eye(2, dtype=complex),
    "X": np.array([[0, 1], [1, 0]], dtype=complex),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=complex),
    "Z": np.array([[1, 0], [0, -1]], dtype=complex),
}
_LOWER = np.array([[0, 1], [0, 0]], dtype=complex)   # |1> -> |0>, annihilation
_RAISE = _LOWER.T.copy()


def _kron_local(factors):
    """factors[j] acts on local qubit j; local basis index = sum bit_j 2^j."""
    out = np.ones((1, 1), dtype=complex)
    for f in factors:                    # qubit 0 ends up least significant
        out = np.kron(f, out)
    return out


def _local_ladder(k: int, j: int, create: bool) -> np.ndarray:
    fac = []
    for m in range(k):
        if m < j:
            fac.append(_PAULI["Z"])
        elif m == j:
            fac.append(_RAISE if create else _LOWER)
        else:
            fac.append(_PAULI["I"])
    return _kron_local(fac)


def _monomial(k: int, ops) -> np.ndarray:
    """ops: sequence of (create?, local qubit), applied as a written product."""
    m = np.eye(2 ** k, dtype=complex)
    for create, j in ops:
        m = m @ _local_ladder(k, j, create)
    return m


def _pauli_expand(mat: np.ndarray, k: int):
    """Return [(letters, coefficient)] with letters[j] on local qubit j."""
    out = []
    for letters in itertools.product("IXYZ", repeat=k):
        ps = _kron_local([_PAULI[c] for c in letters])
        c = np.trace(ps @ mat) / 2 ** k
        if abs(c) > 1e-13:
            assert abs(c.imag) < 1e-12, "Hermitian combination expected"
            out.append(("".join(letters), float(c.real)))
    return out


def _dagger(ops):
    return [(not c, j) for (c, j) in reversed(ops)]


def _herm_pair(k, ops):
    return _monomial(k, ops) + _monomial(k, _dagger(ops))


# ----------------------------------------------------------------------------
# bit-mask helpers (W words of uint64, qubit q -> word q//64 bit q%64)
# ----------------------------------------------------------------------------
_ONE = np.uint64(1)
_ALL = np.uint64(0xFFFFFFFFFFFFFFFF)


def _lowmask(k: np.ndarray) -> np.ndarray:
    k = np.asarray(k, dtype=np.int64)
    kk = np.clip(k, 0, 63).astype(np.uint64)
    m = np.left_shift(_ONE, kk) - _ONE
    return np.where(k >= 64, _ALL, np.where(k <= 0, np.uint64(0), m)).astype(np.uint64)


def _range_mask(lo: np.ndarray, hi: np.ndarray, W: int) -> np.ndarray:
    """[T, W] words with bits lo <= q < hi set (empty if hi <= lo)."""
    lo = np.asarray(lo, dtype=np.int64)
    hi = np.asarray(hi, dtype=np.int64)
    out = np.zeros((lo.size, W), dtype=np.uint64)
    for w in range(W):
        a = np.clip(lo - 64 * w, 0, 64)
        b = np.clip(hi - 64 * w, 0, 64)
        m = _lowmask(b) & ~_lowmask(a)
        out[:, w] = np.where(b > a, m, np.uint64(0))
    return out


def _bit(pos: np.ndarray, W: int) -> np.ndarray:
    pos = np.asarray(pos, dtype=np.int64)
    out = np.zeros((pos.size, W), dtype=np.uint64)
    for w in range(W):
        inw = (pos >= 64 * w) & (pos < 64 * w + 64)
        sh = np.clip(pos - 64 * w, 0, 63).astype(np.uint64)
        out[:, w] = np.where(inw, np.left_shift(_ONE, sh), np.uint64(0))
    return out


@dataclass
class PauliHamiltonian:
    n_qubits: int
    coeff: np.ndarray     # float64 [T]
    xy: np.ndarray        # uint64 [T, W]
    yz: np.ndarray        # uint64 [T, W]

    @property
    def n_words(self) -> int:
        return self.xy.shape[1]

    @property
    def n_terms(self) -> int:
        return self.coeff.size


def _emit(letters_by_pos, positions, zstring, coeffs, W):
    """Assemble terms from local letters at positions [T, k] plus Z string."""
    T = coeffs.size
    xb = np.zeros((T, W), dtype=np.uint64)
    yb = np.zeros((T, W), dtype=np.uint64)
    zb = zstring.copy()
    for j, ch in enumerate(letters_by_pos):
        b = _bit(positions[:, j], W)
        if ch == "X":
            xb |= b
        elif ch == "Y":
            yb |= b
        elif ch == "Z":
            zb |= b
    return coeffs, xb | yb, yb | zb


# ----------------------------------------------------------------------------
# generator
# ----------------------------------------------------------------------------
def jw_hamiltonian(h: np.ndarray, g: np.ndarray, drop: float = 1e-10) -> PauliHamiltonian:
    n = h.shape[0]
    N = 2 * n
    W = (N + 63) // 64
    P = np.arange(N)
    sp = P // 2
    spin = P % 2

    def t(A, B):
        return np.where(spin[A] == spin[B], h[sp[A], sp[B]], 0.0)

    def gso(A, B, C, D):
        ok = (spin[A] == spin[B]) & (spin[C] == spin[D])
        return np.where(ok, g[sp[A], sp[B], sp[C], sp[D]], 0.0)

    def cK(A, B, C, D):
        # coefficient of a+_A a+_B a_D a_C (A<B, C<D) after antisymmetrisation
        return gso(A, C, B, D) - gso(A, D, B, C)

    out_c, out_xy, out_yz = [], [], []

    # --- F empty: number operators ------------------------------------------
    A, B = np.triu_indices(N, 1)
    cab = cK(A, B, A, B)
    tpp = t(P, P)
    const = tpp.sum() / 2 + cab.sum() / 4
    zc = -tpp / 2
    np.add.at(zc, A, -cab / 4)
    np.add.at(zc, B, -cab / 4)
    zero = np.zeros((1, W), dtype=np.uint64)
    out_c.append(np.array([const]))
    out_xy.append(zero)
    out_yz.append(zero)
    out_c.append(zc)
    out_xy.append(np.zeros((N, W), dtype=np.uint64))
    out_yz.append(_bit(P, W))
    out_c.append(cab / 4)
    out_xy.append(np.zeros((A.size, W), dtype=np.uint64))
    out_yz.append(_bit(A, W) | _bit(B, W))

    # --- |F| = 2 --------------------------------------------------------------
    # one-body hopping on local qubits (P, Q)
    hop = _pauli_expand(_herm_pair(2, [(True, 0), (False, 1)]), 2)
    # n_R a+_P a_Q type two-body monomials, three placements of R
    two = {}
    for case in ("R<P", "P<R<Q", "Q<R"):
        loc = {"R<P": (1, 2, 0), "P<R<Q": (0, 2, 1), "Q<R": (0, 1, 2)}[case]
        lp, lq, lr = loc
        cre = sorted((lr, lp))
        ann = sorted((lr, lq))
        # a+_A a+_B a_D a_C with (A,B) = sort(R,P), (C,D) = sort(R,Q)
        ops = [(True, cre[0]), (True, cre[1]), (False, ann[1]), (False, ann[0])]
        two[case] = (loc, _pauli_expand(_herm_pair(3, ops), 3))

    Pp, Qq = np.triu_indices(N, 1)
    same = spin[Pp] == spin[Qq]
    Pp, Qq = Pp[same], Qq[same]
    rows_c, rows_xy, rows_yz, rows_grp = [], [], [], []
    zs = _range_mask(Pp + 1, Qq, W)
    tpq = t(Pp, Qq)
    pos2 = np.stack([Pp, Qq], axis=1)
    gid = np.arange(Pp.size)
    for letters, mult in hop:
        c, xy, yz = _emit(letters, pos2, zs, tpq * mult, W)
        rows_c.append(c); rows_xy.append(xy); rows_yz.append(yz); rows_grp.append(gid)
    for Rv in range(N):
        sel = (Pp != Rv) & (Qq != Rv)
        p_, q_ = Pp[sel], Qq[sel]
        r_ = np.full(p_.size, Rv)
        g_ = gid[sel]
        rp = np.sort(np.stack([r_, p_], 1), 1)
        rq = np.sort(np.stack([r_, q_], 1), 1)
        coef = cK(rp[:, 0], rp[:, 1], rq[:, 0], rq[:, 1])
        for case, (loc, terms) in two.items():
            if case == "R<P":
                m = Rv < p_
            elif case == "Q<R":
                m = Rv > q_
            else:
                m = (Rv > p_) & (Rv < q_)
            if not m.any():
                continue
            pos = np.zeros((m.sum(), 3), dtype=np.int64)
            pos[:, loc[0]] = p_[m]
            pos[:, loc[1]] = q_[m]
            pos[:, loc[2]] = Rv
            zstr = _range_mask(p_[m] + 1, q_[m], W) & ~_bit(np.full(m.sum(), Rv), W)
            for letters, mult in terms:
                c, xy, yz = _emit(letters, pos, zstr, coef[m] * mult, W)
                rows_c.append(c); rows_xy.append(xy); rows_yz.append(yz); rows_grp.append(g_[m])
    c2 = np.concatenate(rows_c)
    xy2 = np.concatenate(rows_xy)
    yz2 = np.concatenate(rows_yz)
    grp = np.concatenate(rows_grp)
    # merge identical strings; order groups by (P, Q) and strings inside a group
    keys = [grp] + [xy2[:, w] for w in range(W)] + [yz2[:, w] for w in range(W)]
    order = np.lexsort(tuple(reversed(keys)))
    srt = np.stack([k[order] for k in keys], axis=1)
    new = np.ones(order.size, dtype=bool)
    new[1:] = np.any(srt[1:] != srt[:-1], axis=1)
    starts = np.flatnonzero(new)
    out_c.append(np.add.reduceat(c2[order], starts))
    out_xy.append(xy2[order][starts])
    out_yz.append(yz2[order][starts])

    # --- |F| = 4 --------------------------------------------------------------
    # local qubits 0<1<2<3; pairings (A,B | C,D)
    pairings = [((0, 1), (2, 3)), ((0, 2), (1, 3)), ((0, 3), (1, 2))]
    exp4 = []
    for (a, b), (c, d) in pairings:
        ops = [(True, a), (True, b), (False, d), (False, c)]
        exp4.append(dict(_pauli_expand(_herm_pair(4, ops), 4)))
    letters4 = sorted(set().union(*[e.keys() for e in exp4]))
    mult4 = np.array([[e.get(s, 0.0) for e in exp4] for s in letters4])   # [S, 3]

    alpha = P[spin == 0]
    beta = P[spin == 1]
    quads = []
    for orb in (alpha, beta):
        cmb = np.array(list(itertools.combinations(range(orb.size), 4)), dtype=np.int64).reshape(-1, 4)
        quads.append(orb[cmb])
    ia, ja = np.triu_indices(alpha.size, 1)
    ib, jb = np.triu_indices(beta.size, 1)
    aa = np.stack([alpha[ia], alpha[ja]], 1)
    bb = np.stack([beta[ib], beta[jb]], 1)
    mix = np.concatenate([np.repeat(aa, bb.shape[0], axis=0), np.tile(bb, (aa.shape[0], 1))], axis=1)
    quads.append(np.sort(mix, axis=1))
    quad = np.concatenate(quads, axis=0)
    quad = quad[np.lexsort(tuple(quad[:, j] for j in (3, 2, 1, 0)))]
    s0, s1, s2, s3 = quad.T
    coefs = np.stack([cK(s0, s1, s2, s3), cK(s0, s2, s1, s3), cK(s0, s3, s1, s2)], axis=1)
    strc = coefs @ mult4.T                                       # [Q, S]
    zq = _range_mask(s0 + 1, s1, W) | _range_mask(s2 + 1, s3, W)
    Qn, S = strc.shape
    xy4 = np.zeros((Qn, S, W), dtype=np.uint64)
    yz4 = np.zeros((Qn, S, W), dtype=np.uint64)
    for si, letters in enumerate(letters4):
        _, xy, yz = _emit(letters, quad, zq, strc[:, si], W)
        xy4[:, si] = xy
        yz4[:, si] = yz
    out_c.append(strc.reshape(-1))
    out_xy.append(xy4.reshape(-1, W))
    out_yz.append(yz4.reshape(-1, W))

    coeff = np.concatenate(out_c)
    xy = np.concatenate(out_xy)
    yz = np.concatenate(out_yz)
    keep = np.abs(coeff) >= drop
    return PauliHamiltonian(N, np.ascontiguousarray(coeff[keep]),
                            np.ascontiguousarray(xy[keep]), np.ascontiguousarray(yz[keep]))


def random_jw(n_qubits: int, rng: np.random.Generator) -> tuple[PauliHamiltonian, np.ndarray, np.ndarray]:
    assert n_qubits % 2 == 0, "spin orbitals come in alpha/beta pairs"
    h, g = spatial_integrals(n_qubits // 2, rng)
    return jw_hamiltonian(h, g), h, g


def random_pauli(n_qubits: int, n_terms: int, rng: np.random.Generator,
                 max_flip: int | None = None) -> PauliHamiltonian:
    """Random Pauli strings with all four letters (odd |Y| included) and
    N(0,1) coefficients; used where no chemistry structure is wanted."""
    W = (n_qubits + 63) // 64
    letters = rng.integers(0, 4, size=(n_terms, n_qubits))   # 0 I 1 X 2 Y 3 Z
    if max_flip is not None:
        for t_ in range(n_terms):
            flips = np.flatnonzero((letters[t_] == 1) | (letters[t_] == 2))
            if flips.size > max_flip:
                drop_ = rng.choice(flips, size=flips.size - max_flip, replace=False)
                letters[t_, drop_] = rng.choice([0, 3], size=drop_.size)
    xy = np.zeros((n_terms, W), dtype=np.uint64)
    yz = np.zeros((n_terms, W), dtype=np.uint64)
    for q in range(n_qubits):
        b = np.uint64(1) << np.uint64(q % 64)
        l = letters[:, q]
        xy[(l == 1) | (l == 2), q // 64] |= b
        yz[(l == 2) | (l == 3), q // 64] |= b
    return PauliHamiltonian(n_qubits, rng.normal(size=n_terms), xy, yz)
