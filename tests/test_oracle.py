"""Pins of the CPU oracle against facts fixed outside it.

Each test checks the oracle against something it does not compute itself:
values printed in the paper's toy problem, the textbook 2x2 Pauli matrices,
a second-quantised build of H, the Slater-Condon closed form, an exact
eigenvector, the Rayleigh quotient and its variance, finite differences and
torch autograd over a dense formulation.
"""
import json
from pathlib import Path

import numpy as np
import pytest

import oracle
import pins
from synth import jw, samples

GOLDEN = Path(__file__).resolve().parent / "golden"


def _mask(bitstring):
    """Paper bit strings put qubit 0 first."""
    return sum(1 << q for q, ch in enumerate(bitstring) if ch == "1")


def _toy_inputs():
    d = json.loads((GOLDEN / "toy_model.json").read_text())
    coeff = np.array([t["coeff"] for t in d["terms"]])
    xy = np.array([[_mask(t["XY"])] for t in d["terms"]], dtype=np.uint64)
    yz = np.array([[_mask(t["YZ"])] for t in d["terms"]], dtype=np.uint64)
    for t in d["terms"]:   # the printed masks agree with the printed Pauli strings
        ls = t["pauli"]
        assert t["XY"] == "".join("1" if c in "XY" else "0" for c in ls)
        assert t["YZ"] == "".join("1" if c in "YZ" else "0" for c in ls)
        assert t["Y"] == "".join("1" if c == "Y" else "0" for c in ls)
    ham = jw.PauliHamiltonian(4, coeff, xy, yz)
    keys = np.array([[_mask(s)] for s in d["samples"]], dtype=np.uint64)
    logpsi = np.log(np.array(d["psi"], dtype=complex))
    return d, ham, keys, logpsi


def test_toy_unique_xy_and_term_sets():
    d, ham, keys, logpsi = _toy_inputs()
    g = oracle.groups(ham)
    want = np.zeros(ham.n_terms, dtype=np.int64)
    for gi, members in enumerate(d["term_sets"]):
        want[members] = gi
    assert g.tolist() == want.tolist()
    for gi, s in enumerate(d["unique_xy"]):
        assert int(ham.xy[np.flatnonzero(g == gi)[0], 0]) == _mask(s)


def test_toy_pairs_elements_energies():
    d, ham, keys, logpsi = _toy_inputs()
    pi, pj, pg, hij = oracle.find_pairs(ham, keys, with_elements=True)
    coupled = [pj[pi == i].tolist() for i in range(3)]
    assert coupled == d["coupled"]
    # row-major canonical order: the fourth pair's x is x_1
    assert pi[3] == d["pointer_example"]["x_ptr_3"]
    got = {(int(a), int(b)): h for a, b, h in zip(pi, pj, hij)}
    assert len(got) == len(d["matrix_elements"])
    for m in d["matrix_elements"]:
        assert abs(got[(m["i"], m["j"])] - m["h"]) < 1e-12
    # the group of each pair is the unique XY equal to x ^ x'
    xs = [_mask(s) for s in d["unique_xy"]]
    for a, b, g in zip(pi, pj, pg):
        assert int(keys[a, 0] ^ keys[b, 0]) == xs[g]
    e = oracle.local_energy(ham, keys, logpsi)
    np.testing.assert_allclose(e.real, d["local_energy"], atol=1e-12)
    np.testing.assert_allclose(e.imag, 0.0, atol=1e-12)


def _dense_eloc(H, basis_idx, logpsi):
    sub = H[np.ix_(basis_idx, basis_idx)]
    psi = np.exp(logpsi)
    return (sub @ psi) / psi


@pytest.mark.parametrize("N,T,seed", [(3, 20, 0), (5, 60, 1), (6, 120, 2), (8, 200, 3)])
def test_dense_random_pauli(N, T, seed):
    """All four letters, odd |Y| included: fixes the i^|Y| factor and that the
    phase is evaluated on the ket x'."""
    rng = np.random.default_rng(seed)
    ham = jw.random_pauli(N, T, rng)
    H = pins.dense_pauli_kron(ham)
    M = min(2 ** N, 40)
    basis = np.sort(rng.choice(2 ** N, size=M, replace=False))
    keys = rng.permutation(basis).astype(np.uint64)[:, None]
    logpsi = rng.normal(size=M) + 1j * rng.uniform(0, 2 * np.pi, size=M)
    e = oracle.local_energy(ham, keys, logpsi)
    np.testing.assert_allclose(e, _dense_eloc(H, keys[:, 0].astype(np.int64), logpsi), atol=1e-10, rtol=1e-10)
    # every matrix element of H between sampled states, coupled or not
    ii, jj = np.meshgrid(np.arange(M), np.arange(M), indexing="ij")
    me = oracle.matrix_elements(ham, keys[ii.ravel()], keys[jj.ravel()])
    np.testing.assert_allclose(me, H[keys[ii.ravel(), 0].astype(np.int64), keys[jj.ravel(), 0].astype(np.int64)],
                               atol=1e-12)


@pytest.mark.parametrize("N,T,seed,max_flip", [(3, 20, 10, None), (5, 60, 11, 2), (7, 90, 12, 2)])
def test_phase_exponents_against_kron(N, T, seed, max_flip):
    """Each exponent k the oracle gives for a term of a pair's group is that
    term's own matrix element i^k, read from the Kronecker product of the
    textbook 2x2 matrices (odd |Y| included); the terms come in ascending
    caller index, and uncoupled pairs get none."""
    rng = np.random.default_rng(seed)
    ham = jw.random_pauli(N, T, rng, max_flip=max_flip)
    D = 2 ** N
    ii, jj = np.meshgrid(np.arange(D), np.arange(D), indexing="ij")
    x = ii.ravel().astype(np.uint64)[:, None]
    xp = jj.ravel().astype(np.uint64)[:, None]
    off, k = oracle.phase_exponents(ham, x, xp)
    mats = [pins.dense_pauli_kron(jw.PauliHamiltonian(N, np.ones(1), ham.xy[l:l + 1], ham.yz[l:l + 1]))
            for l in range(T)]
    xy = ham.xy[:, 0].astype(np.int64)
    ipow = np.array([1, 1j, -1, -1j])
    checked = 0
    for p in range(D * D):
        a, b = int(x[p, 0]), int(xp[p, 0])
        terms = np.flatnonzero(xy == (a ^ b))
        ks = k[off[p]:off[p + 1]]
        assert ks.size == terms.size
        for l, kk in zip(terms, ks):
            assert mats[l][a, b] == ipow[kk], (p, l, kk)
            checked += 1
    assert checked == int(off[-1]) > 0


def test_dense_builds_agree():
    ham = jw.random_pauli(5, 40, np.random.default_rng(9))
    np.testing.assert_allclose(pins.dense_pauli(ham), pins.dense_pauli_kron(ham), atol=1e-13)


@pytest.mark.parametrize("N", [4, 6, 8])
def test_jw_generator_against_second_quantisation(N):
    ham, h, g = jw.random_jw(N, np.random.default_rng(100 + N))
    Hf = pins.dense_fermion(h, g)
    Hp = pins.dense_pauli(ham)
    np.testing.assert_allclose(Hp, Hf, atol=1e-12)
    # the oracle on U = the whole Fock space reproduces H psi / psi
    rng = np.random.default_rng(N)
    keys = rng.permutation(2 ** N).astype(np.uint64)[:, None]
    logpsi = rng.normal(scale=0.5, size=2 ** N) + 1j * rng.uniform(0, 2 * np.pi, size=2 ** N)
    e = oracle.local_energy(ham, keys, logpsi)
    np.testing.assert_allclose(e, _dense_eloc(Hf, keys[:, 0].astype(np.int64), logpsi), atol=1e-10)


@pytest.mark.parametrize("N,ne", [(12, 6), (28, 14), (52, 20), (100, 30)])
def test_single_determinant_slater_condon(N, ne):
    """U = {x}: E_loc = E^var = H_xx, the Slater-Condon energy of x."""
    rng = jw.rng_for(1000 + N, 0)
    h, g = jw.spatial_integrals(N // 2, rng)
    ham = jw.jw_hamiltonian(h, g)
    keys, _ = samples.excitation_batch(N, ne, 6 if N < 100 else 2, jw.rng_for(1000 + N, 1))
    for k in keys:
        occ = pins.occupied_modes(k, N)
        ref = pins.slater_condon(h, g, occ)
        e = oracle.local_energy(ham, k[None, :], np.array([0.3 + 1.1j]))
        assert abs(e[0] - ref) < 1e-9 * max(1.0, abs(ref))
        E, var, tot = oracle.energy(e, np.array([0.3 + 1.1j]))
        assert abs(E - ref) < 1e-9 * max(1.0, abs(ref)) and abs(var) < 1e-18


def _sector(N, na, nb):
    import itertools
    out = []
    for ca in itertools.combinations(range(0, N, 2), na):
        for cb in itertools.combinations(range(1, N, 2), nb):
            out.append(sum(1 << q for q in ca + cb))
    return np.array(sorted(out), dtype=np.int64)


def test_eigenvector_gives_constant_local_energy(small_workload):
    """U = a whole (n_alpha, n_beta) sector is invariant under H, so for an
    eigenvector psi every E_loc^var(x) equals the eigenvalue and Var = 0."""
    w = small_workload
    basis = _sector(12, 3, 3)
    Hs = pins.dense_fermion(w.h, w.g, basis=basis)
    lam, vec = np.linalg.eigh(Hs)
    for k in (0, 7):
        psi = vec[:, k]
        assert np.abs(psi).min() > 1e-10
        rng = np.random.default_rng(k)
        order = rng.permutation(basis.size)
        keys = basis[order].astype(np.uint64)[:, None]
        logpsi = np.log(psi[order].astype(complex))
        e = oracle.local_energy(w.ham, keys, logpsi)
        np.testing.assert_allclose(e, lam[k], atol=1e-9)
        E, var, _ = oracle.energy(e, logpsi)
        assert abs(E - lam[k]) < 1e-10 and var < 1e-16


def test_energy_is_rayleigh_quotient_and_variance(small_workload):
    """With |psi|^2 weights, E^var = <psi|H_UU|psi>/<psi|psi> and
    Var = ||H_UU psi||^2/||psi||^2 - |E|^2; E^var >= the lowest eigenvalue."""
    w = small_workload
    H = pins.dense_pauli(w.ham)
    idx = w.keys[:, 0].astype(np.int64)
    Huu = H[np.ix_(idx, idx)]
    psi = np.exp(w.logpsi)
    nrm = np.vdot(psi, psi).real
    Eref = np.vdot(psi, Huu @ psi) / nrm
    Vref = np.vdot(Huu @ psi, Huu @ psi).real / nrm - abs(Eref) ** 2
    e = oracle.local_energy(w.ham, w.keys, w.logpsi)
    E, var, tot = oracle.energy(e, w.logpsi)
    assert abs(E - Eref) < 1e-10
    assert abs(E.imag) < 1e-10
    assert abs(var - Vref) < 1e-8 * max(1.0, Vref)
    np.testing.assert_allclose(tot, nrm, rtol=1e-12)
    assert E.real >= np.linalg.eigvalsh(Huu)[0] - 1e-10


def test_counts_weighting():
    """Eq. energy_estimator_via_unique: sum E_loc n / N_s."""
    d, ham, keys, logpsi = _toy_inputs()
    e = oracle.local_energy(ham, keys, logpsi)
    n = np.array([5.0, 2.0, 1.0])
    E, var, tot = oracle.energy(e, logpsi, n)
    assert abs(E - (0.8 * 5 + 0.6 * 2 + 1.4 * 1) / 8) < 1e-12
    assert tot == 8.0
    ref_var = (5 * (0.8 - E.real) ** 2 + 2 * (0.6 - E.real) ** 2 + (1.4 - E.real) ** 2) / 8
    assert abs(var - ref_var) < 1e-12


def test_pairs_symmetric_hermitian_and_sector(small_workload):
    w = small_workload
    pi, pj, pg, hij = oracle.find_pairs(w.ham, w.keys, with_elements=True)
    fwd = {(int(a), int(b)): h for a, b, h in zip(pi, pj, hij)}
    for (a, b), h in fwd.items():
        assert (b, a) in fwd
        assert abs(fwd[(b, a)] - np.conj(h)) < 1e-12
    # pairs are row-major sorted and unique
    key = pi.astype(np.int64) * w.n_unique + pj
    assert np.all(np.diff(key) > 0)
    # particle number and S_z: a coupled pair across sectors has H = 0
    bits = samples.bits_from_key(w.keys, 12)
    na = bits[:, 0::2].sum(1)
    nb = bits[:, 1::2].sum(1)
    scale = np.abs(w.ham.coeff).sum()
    cross = (na[pi] != na[pj]) | (nb[pi] != nb[pj])
    assert cross.any(), "the small workload has cross-sector XOR pairs"
    assert np.abs(hij[cross]).max() <= 1e-12 * scale


def test_bit_permutation_invariance(small_workload):
    w = small_workload
    perm = np.random.default_rng(5).permutation(12)

    def permute(a):
        out = np.zeros_like(a)
        for q in range(12):
            out[:, 0] |= ((a[:, 0] >> np.uint64(q)) & np.uint64(1)) << np.uint64(perm[q])
        return out
    ham2 = jw.PauliHamiltonian(12, w.ham.coeff, permute(w.ham.xy), permute(w.ham.yz))
    e1 = oracle.local_energy(w.ham, w.keys, w.logpsi)
    e2 = oracle.local_energy(ham2, permute(w.keys), w.logpsi)
    np.testing.assert_allclose(e1, e2, atol=1e-11)
    p1 = oracle.find_pairs(w.ham, w.keys)
    p2 = oracle.find_pairs(ham2, permute(w.keys))
    for a, b in zip(p1, p2):
        np.testing.assert_array_equal(a, b)


def test_term_order_only_relabels_groups(small_workload):
    w = small_workload
    perm = np.random.default_rng(3).permutation(w.ham.n_terms)
    ham2 = jw.PauliHamiltonian(12, w.ham.coeff[perm], w.ham.xy[perm], w.ham.yz[perm])
    np.testing.assert_allclose(oracle.local_energy(ham2, w.keys, w.logpsi),
                               oracle.local_energy(w.ham, w.keys, w.logpsi), atol=1e-11)


def test_duplicate_keys_rejected():
    d, ham, keys, logpsi = _toy_inputs()
    with pytest.raises(oracle.OracleError):
        oracle.local_energy(ham, np.concatenate([keys, keys[:1]]), np.concatenate([logpsi, logpsi[:1]]))


# ----------------------------------------------------------------------------
# adjoint
# ----------------------------------------------------------------------------
def _energy_of(ham, keys, L, weights):
    e = oracle.local_energy(ham, keys, L)
    E, _, _ = oracle.energy(e, L, weights)
    return E


@pytest.mark.parametrize("use_counts", [False, True])
def test_adjoint_finite_differences(small_workload, use_counts):
    w = small_workload
    rng = np.random.default_rng(11)
    weights = rng.integers(1, 20, size=w.n_unique).astype(float) if use_counts else None
    L = w.logpsi
    e = oracle.local_energy(w.ham, w.keys, L)
    E, _, _ = oracle.energy(e, L, weights)
    ys = rng.choice(w.n_unique, size=12, replace=False)
    h = 1e-6
    for grad_e, part in ((1.0, "re"), (1j, "im")):
        g = oracle.adjoint(w.ham, w.keys, L, e, grad_e, weights=weights, energy_value=E)
        for y in ys:
            fd = []
            for dv in (1.0, 1j):
                Lp = L.copy(); Lp[y] += h * dv
                Lm = L.copy(); Lm[y] -= h * dv
                Ep = _energy_of(w.ham, w.keys, Lp, weights)
                Em = _energy_of(w.ham, w.keys, Lm, weights)
                dE = (Ep - Em) / (2 * h)
                fd.append(dE.real if part == "re" else dE.imag)
            ref = fd[0] + 1j * fd[1]
            assert abs(g[y] - ref) < 1e-6 * max(1.0, abs(ref)), (y, g[y], ref)
        if use_counts:
            # constant shift of every log psi leaves E unchanged
            assert abs(g.sum()) < 1e-9 * np.abs(g).sum()


def test_adjoint_matches_torch_autograd_dense():
    """Dense torch formulation, E(L) = sum_x w~_x sum_x' H_xx' e^(L_x' - L_x),
    differentiated by torch: fixes the complex-gradient convention."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    N = 6
    ham = jw.random_pauli(N, 80, rng)
    H = pins.dense_pauli_kron(ham)
    M = 30
    basis = rng.choice(2 ** N, size=M, replace=False)
    keys = basis.astype(np.uint64)[:, None]
    L = rng.normal(scale=0.7, size=M) + 1j * rng.uniform(0, 2 * np.pi, size=M)
    Huu = torch.tensor(H[np.ix_(basis, basis)])
    for weights in (None, rng.integers(1, 9, size=M).astype(float)):
        for grad_e in (1.0, 1j, 0.3 - 0.8j):
            Lt = torch.tensor(L, requires_grad=True)
            psi = torch.exp(Lt)
            eloc = (Huu @ psi) / psi
            if weights is None:
                wt = torch.exp(2 * Lt.real)
            else:
                wt = torch.tensor(weights)
            wt = wt / wt.sum()
            E = (wt * eloc).sum()
            ge = complex(grad_e)
            loss = ge.real * E.real + ge.imag * E.imag
            loss.backward()
            e = oracle.local_energy(ham, keys, L)
            Eo, _, _ = oracle.energy(e, L, weights)
            g = oracle.adjoint(ham, keys, L, e, ge, weights=weights, energy_value=Eo)
            np.testing.assert_allclose(g, Lt.grad.numpy(), atol=1e-10)


# ----------------------------------------------------------------------------
# Conventional local energy (Eq. local_energy, the sum over every x'): the
# states outside U with a non-zero matrix element, and E_loc over U and them.
def _dense_misses(H, basis_idx, thresh=1e-9):
    """x' not in U with |<x|H|x'>| > thresh for some x in U (dense H)."""
    rows = np.abs(H[basis_idx, :]).max(axis=0) > thresh
    rows[basis_idx] = False
    return np.flatnonzero(rows)


@pytest.mark.parametrize("N,T,seed", [(5, 40, 20), (7, 80, 21)])
def test_full_local_energy_dense_random_pauli(N, T, seed):
    """Against the dense matrix of textbook Pauli products: the miss set is
    every state outside U that H reaches from U, and E_loc(x) = (H psi)(x) /
    psi(x) over the whole space for a random psi."""
    rng = np.random.default_rng(seed)
    ham = jw.random_pauli(N, T, rng, max_flip=3)
    H = pins.dense_pauli_kron(ham)
    D = 2 ** N
    M = 12
    idx = rng.choice(D, size=M, replace=False)
    keys = idx.astype(np.uint64)[:, None]
    V = oracle.find_misses(ham, keys)
    np.testing.assert_array_equal(V[:, 0].astype(np.int64), _dense_misses(H, idx))
    L = rng.normal(scale=0.5, size=D) + 1j * rng.uniform(0, 2 * np.pi, size=D)
    psi = np.exp(L)
    vi = V[:, 0].astype(np.int64)
    e = oracle.local_energy_full(ham, keys, L[idx], V, L[vi])
    np.testing.assert_allclose(e, (H @ psi)[idx] / psi[idx], rtol=1e-10, atol=1e-10)


def test_full_local_energy_jw_cancellation():
    """Jordan-Wigner H of real integrals: strings coupling different
    particle-number sectors cancel, so those x' are not misses even though
    x ^ x' is an XY mask of H; the miss set equals the dense non-zeros."""
    N = 8
    rng = np.random.default_rng(30)
    ham, h, g = jw.random_jw(N, rng)
    H = pins.dense_pauli(ham)
    sector = _sector(N, 2, 2)
    others = np.setdiff1d(np.arange(2 ** N), sector)
    idx = np.concatenate([rng.choice(sector, size=10, replace=False), rng.choice(others, size=6, replace=False)])
    keys = idx.astype(np.uint64)[:, None]
    V = oracle.find_misses(ham, keys)
    np.testing.assert_array_equal(V[:, 0].astype(np.int64), _dense_misses(H, idx))
    # some XOR partners of U exist that are not coupled (cancelled strings)
    xy = {int(m) for m in ham.xy[:, 0]}
    partners = {int(x) ^ m for x in idx for m in xy} - set(int(x) for x in idx)
    assert len(partners) > V.shape[0]
    L = rng.normal(scale=0.5, size=2 ** N) + 1j * rng.uniform(0, 2 * np.pi, size=2 ** N)
    psi = np.exp(L)
    e = oracle.local_energy_full(ham, keys, L[idx], V, L[V[:, 0].astype(np.int64)])
    np.testing.assert_allclose(e, (H @ psi)[idx] / psi[idx], rtol=1e-10, atol=1e-10)
    # without the misses' amplitudes the conventional sum is incomplete
    with pytest.raises(oracle.OracleError):
        oracle.local_energy_full(ham, keys, L[idx], V[:-1], L[V[:-1, 0].astype(np.int64)])


@pytest.mark.parametrize("k", [0, 5])
def test_full_local_energy_of_eigenvector_is_eigenvalue(k):
    """For an eigenvector psi of H, E_loc(x) = lambda for every x, whatever
    U is (no sector structure in a random Pauli Hamiltonian)."""
    rng = np.random.default_rng(40 + k)
    N = 6
    ham = jw.random_pauli(N, 50, rng, max_flip=3)
    H = pins.dense_pauli_kron(ham)
    lam, vec = np.linalg.eigh(H)
    psi = vec[:, k]
    assert np.abs(psi).min() > 1e-8
    L = np.log(psi.astype(complex))
    idx = rng.choice(2 ** N, size=9, replace=False)
    keys = idx.astype(np.uint64)[:, None]
    V = oracle.find_misses(ham, keys)
    e = oracle.local_energy_full(ham, keys, L[idx], V, L[V[:, 0].astype(np.int64)])
    np.testing.assert_allclose(e, lam[k], atol=1e-9)


def test_misses_two_words_brute_force():
    """70 qubits (two words per key): the miss set equals a brute force over
    U x Pauli strings whose matrix elements are products of textbook 2x2
    entries, sorted as 128-bit integers (high word first)."""
    rng = np.random.default_rng(50)
    N, T, M = 70, 40, 25
    ham = jw.random_pauli(N, T, rng, max_flip=2)
    keys = np.unique(rng.integers(0, 2 ** 63, size=(M, 2), dtype=np.int64).astype(np.uint64), axis=0)
    keys[:, 1] &= np.uint64((1 << (N - 64)) - 1)
    keys = np.unique(keys, axis=0)
    U = {(int(k[1]) << 64) | int(k[0]) for k in keys}
    lets = [pins.letters(N, ham.xy[l], ham.yz[l]) for l in range(T)]

    def entry(ls, x, xp):
        v = 1.0 + 0j
        for q in range(N):
            v *= pins.PAULI[ls[q]][(x >> q) & 1, (xp >> q) & 1]
            if v == 0:
                return 0j
        return v

    masks = {}
    for l in range(T):
        m = (int(ham.xy[l, 1]) << 64) | int(ham.xy[l, 0])
        masks.setdefault(m, []).append(l)
    want = set()
    for x in U:
        for m, ls in masks.items():
            xp = x ^ m
            if xp in U:
                continue
            h = sum(ham.coeff[l] * entry(lets[l], x, xp) for l in ls)
            if abs(h) > 1e-10 * sum(abs(ham.coeff[l]) for l in ls):
                want.add(xp)
    V = oracle.find_misses(ham, keys)
    got = [(int(v[1]) << 64) | int(v[0]) for v in V]
    assert got == sorted(want)
