"""Parity of the HIP engine (through the C ABI) with the CPU oracle.

Bars: coupled pairs and group ids bit-exact; FP64 local energies within
1e-9 Ha (the oracle and the kernels differ only in summation order; the
observed gap is ~1e-13); the compensated FP32 form within 1e-6 Ha, the
tolerance the accuracy target of the method states.
"""
import json
from pathlib import Path

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from synth import configs, jw, samples  # noqa: E402

TOL64 = 1e-9
TOL32 = 1e-6


@pytest.fixture(scope="module")
def eng():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2408_07625_amd as pe
    e = pe.Engine(0)
    yield e
    e.close()


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def keys_dev(keys):
    return dev(keys.view(np.int64))


def load(eng, ham, keys):
    eng.set_hamiltonian(ham.n_qubits, ham.coeff, ham.xy, ham.yz)
    eng.set_samples(keys_dev(keys))


def oracle_pairs(ham, keys, rows=None):
    pi, pj, pg = oracle.find_pairs(ham, keys, rows=rows)
    return pi.astype(np.int64), pj.astype(np.int64), pg.astype(np.int64)


def gpu_pairs(eng, variant):
    i, j, g = eng.find_pairs(variant)
    return i.cpu().numpy().astype(np.int64), j.cpu().numpy().astype(np.int64), g.cpu().numpy().astype(np.int64)


# ----------------------------------------------------------------------------
def _toy():
    d = json.loads((Path(__file__).resolve().parent / "golden" / "toy_model.json").read_text())

    def m(s):
        return sum(1 << q for q, ch in enumerate(s) if ch == "1")
    ham = jw.PauliHamiltonian(4, np.array([t["coeff"] for t in d["terms"]]),
                              np.array([[m(t["XY"])] for t in d["terms"]], dtype=np.uint64),
                              np.array([[m(t["YZ"])] for t in d["terms"]], dtype=np.uint64))
    keys = np.array([[m(s)] for s in d["samples"]], dtype=np.uint64)
    return d, ham, keys, np.log(np.array(d["psi"], dtype=complex))


@pytest.mark.parametrize("variant", ["terms", "batch", "trie"])
@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_toy_model(eng, variant, precision):
    d, ham, keys, logpsi = _toy()
    load(eng, ham, keys)
    e, st = eng.local_energy(dev(logpsi), variant=variant, precision=precision)
    np.testing.assert_allclose(e.cpu().numpy(), d["local_energy"], atol=1e-12)
    i, j, g = gpu_pairs(eng, variant)
    assert [j[i == r].tolist() for r in range(3)] == d["coupled"]
    assert g.tolist() == [0, 2, 1, 2, 0, 1, 0]
    h = eng.pair_elements(dev(i, torch.int32), dev(j, torch.int32)).cpu().numpy()
    want = {(m["i"], m["j"]): m["h"] for m in d["matrix_elements"]}
    np.testing.assert_allclose(h, [want[(a, b)] for a, b in zip(i, j)], atol=1e-12)


# ----------------------------------------------------------------------------
def check_workload(eng, w, variants=("terms", "batch", "trie"), rows=None, pairs=True):
    load(eng, w.ham, w.keys)
    M = w.n_unique
    L = dev(w.logpsi)
    W8 = None if w.weights is None else dev(w.weights)
    if rows is None:
        ref = oracle.local_energy(w.ham, w.keys, w.logpsi)
        sel = np.arange(M)
    else:
        ref = np.concatenate([oracle.local_energy(w.ham, w.keys, w.logpsi, rows=r) for r in rows])
        sel = np.concatenate([np.arange(a, b) for a, b in rows])
    for variant in variants:
        for prec, tol in (("fp64", TOL64), ("fp32c", TOL32)):
            e, st = eng.local_energy(L, W8, variant=variant, precision=prec)
            got = e.cpu().numpy()[sel]
            err = np.abs(got - ref).max()
            print(f"{w.name} {variant} {prec}: max |dE_loc| = {err:.3e}")
            assert err <= tol, (variant, prec, err)
            if rows is None:
                E, var, tot = oracle.energy(ref, w.logpsi, w.weights)
                s = st.cpu().numpy()
                assert abs(s[0] - E.real) <= tol and abs(s[1] - E.imag) <= tol
                assert abs(s[2] - var) <= tol * max(1.0, var)
                np.testing.assert_allclose(s[3], tot, rtol=1e-12)
    if pairs:
        if rows is None:
            ref_p = oracle_pairs(w.ham, w.keys)
            for variant in variants:
                got_p = gpu_pairs(eng, variant)
                for a, b in zip(got_p, ref_p):
                    np.testing.assert_array_equal(a, b)
        else:
            for variant in variants:
                got_p = gpu_pairs(eng, variant)
                for (a, b) in rows:
                    ref_p = oracle_pairs(w.ham, w.keys, rows=(a, b))
                    m = (got_p[0] >= a) & (got_p[0] < b)
                    for x, y in zip(got_p, ref_p):
                        np.testing.assert_array_equal(x[m], y)


def test_small_workload(eng, small_workload):
    check_workload(eng, small_workload)


def test_medium_workload(eng, medium_workload):
    w = medium_workload
    check_workload(eng, w, rows=[(0, 700), (31000, 31333), (65536 - 517, 65536)])
    # full-row energies, the configuration the benchmark times
    ref = oracle.local_energy(w.ham, w.keys, w.logpsi)
    e, st = eng.local_energy(dev(w.logpsi), variant="terms", precision="fp64")
    assert np.abs(e.cpu().numpy() - ref).max() <= TOL64
    E, var, tot = oracle.energy(ref, w.logpsi)
    s = st.cpu().numpy()
    assert abs(s[0] - E.real) <= TOL64 and abs(s[2] - var) <= TOL64 * max(1.0, var)
    _, npairs = oracle.local_energy(w.ham, w.keys, w.logpsi, rows=(0, w.n_unique), with_pairs=True)
    assert eng.count_pairs("terms") == int(npairs.sum())


# ----------------------------------------------------------------------------
# 52 qubits, 2^20 samples: every variant against the oracle's stored results
# (tests/golden/make_large_golden.py): E_loc, pair count and pair digest of
# 12 800 sampled rows, E and Var over all rows, the total pair count.
GOLDEN = Path(__file__).resolve().parent / "golden"


@pytest.fixture(scope="module")
def large_golden(large_workload):
    import hashlib
    path = GOLDEN / "large_oracle.npz"
    if not path.exists():
        pytest.fail(f"{path} missing: run tests/golden/make_large_golden.py")
    g = dict(np.load(path, allow_pickle=False))
    w = large_workload
    h = hashlib.sha256()
    for a in (w.ham.coeff, w.ham.xy, w.ham.yz, w.keys, w.logpsi):
        h.update(np.ascontiguousarray(a).tobytes())
    assert np.frombuffer(h.digest(), dtype=np.uint8).tobytes() == g["fingerprint"].tobytes(), \
        "the generated 52-qubit inputs differ from those the golden file was made from"
    return g


def gpu_row_digests(eng, variant, rows):
    """(count, digest) of the sampled rows from the engine's canonical pair
    list (sorted by row, so each contiguous block of rows is one slice)."""
    from digest import row_digests
    i, j, g = eng.find_pairs(variant)
    cnt, dig = [], []
    starts = np.flatnonzero(np.diff(rows, prepend=-2) != 1)
    ends = np.append(starts[1:], rows.size)
    for s0, s1 in zip(starts, ends):
        a, b = int(rows[s0]), int(rows[s1 - 1]) + 1
        lo, hi = torch.searchsorted(i, torch.tensor([a, b], dtype=torch.int32, device=i.device)).tolist()
        c, d = row_digests(i[lo:hi].cpu().numpy(), j[lo:hi].cpu().numpy(), g[lo:hi].cpu().numpy(),
                           rows[s0:s1])
        cnt.append(c)
        dig.append(d)
    del i, j, g
    return np.concatenate(cnt), np.concatenate(dig)


@pytest.mark.parametrize("variant", ["terms", "batch", "trie"])
def test_large_workload_golden(eng, large_workload, large_golden, variant):
    w, gold = large_workload, large_golden
    load(eng, w.ham, w.keys)
    rows = gold["rows"]
    L = dev(w.logpsi)
    E_ref = gold["stats"][0] + 1j * gold["stats"][1]
    var_ref = gold["stats"][2]
    for prec, tol in (("fp64", TOL64), ("fp32c", TOL32)):
        e, st = eng.local_energy(L, None, variant=variant, precision=prec)
        err = np.abs(e.cpu().numpy()[rows] - gold["eloc"]).max()
        s = st.cpu().numpy()
        print(f"large {variant} {prec}: max |dE_loc| = {err:.3e}, |dE| = {abs(s[0] + 1j * s[1] - E_ref):.3e}, "
              f"|dVar| = {abs(s[2] - var_ref):.3e}", flush=True)
        assert err <= tol
        assert abs(s[0] - E_ref.real) <= tol and abs(s[1] - E_ref.imag) <= tol
        assert abs(s[2] - var_ref) <= tol * max(1.0, var_ref)
        np.testing.assert_allclose(s[3], gold["stats"][3], rtol=1e-12)
    assert eng.count_pairs(variant) == int(gold["total_pairs"])
    cnt, dig = gpu_row_digests(eng, variant, rows)
    np.testing.assert_array_equal(cnt, gold["count"])
    np.testing.assert_array_equal(dig, gold["digest"])


# ----------------------------------------------------------------------------
WIDE_ROWS = [(0, 100), ((1 << 18) - 77, 1 << 18)]


@pytest.mark.parametrize("variant", ["terms", "batch"])
def test_wide_workload_sampled(eng, wide_workload, variant):
    """100 qubits, two words per key, occurrence-count weights: forward and
    adjoint (the pairs found again by the variant's kernels) on sampled rows."""
    w = wide_workload
    check_workload(eng, w, variants=(variant,), rows=WIDE_ROWS, pairs=False)
    L = dev(w.logpsi)
    Wt = dev(w.weights)
    e, st = eng.local_energy(L, Wt, variant=variant, precision="fp64")
    E = complex(st[0].item(), st[1].item())
    for prec, tol in (("fp64", TOL64), ("fp32c", TOL32)):
        g = eng.adjoint(L, e, st, 1.0 + 0.5j, Wt, variant=variant, precision=prec).cpu().numpy()
        for a, b in WIDE_ROWS:
            ref_e = oracle.local_energy(w.ham, w.keys, w.logpsi, rows=(a, b))
            ref = oracle.adjoint(w.ham, w.keys, w.logpsi, ref_e, 1.0 + 0.5j, weights=w.weights,
                                 energy_value=E, rows=(a, b))
            err = np.abs(g[a:b] - ref).max()
            print(f"wide {variant} adjoint {prec}: max |dG| = {err:.3e} (max |G| {np.abs(ref).max():.3e})")
            assert err <= tol * max(1.0, np.abs(ref).max())


def test_wide_workload_pairs_sampled(eng, wide_workload):
    """Two-word keys: LoopOverBatch's pair list equals the oracle's on the
    sampled rows (row sets of the canonical list)."""
    w = wide_workload
    load(eng, w.ham, w.keys)
    got = gpu_pairs(eng, "batch")
    for a, b in WIDE_ROWS:
        ref = oracle_pairs(w.ham, w.keys, rows=(a, b))
        m = (got[0] >= a) & (got[0] < b)
        for x, y in zip(got, ref):
            np.testing.assert_array_equal(x[m], y)


# ----------------------------------------------------------------------------
@pytest.mark.parametrize("M", [1, 2, 63, 64, 65, 255, 257, 1000])
def test_ragged_batch_sizes(eng, small_workload, M):
    w = small_workload
    keys = w.keys[:M].copy()
    lp = w.logpsi[:M].copy()
    load(eng, w.ham, keys)
    ref = oracle.local_energy(w.ham, keys, lp)
    for variant in ("terms", "batch", "trie"):
        e, st = eng.local_energy(dev(lp), variant=variant)
        assert np.abs(e.cpu().numpy() - ref).max() <= TOL64
        got = gpu_pairs(eng, variant)
        for a, b in zip(got, oracle_pairs(w.ham, keys)):
            np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("chunks,rows", [(1, 8), (3, 4), (17, 8)])
def test_chunking_does_not_change_pairs(eng, small_workload, chunks, rows):
    w = small_workload
    load(eng, w.ham, w.keys)
    ref = oracle.local_energy(w.ham, w.keys, w.logpsi)
    for sig in (True, False):
        eng.set_tuning(chunks, sig, rows)
        try:
            for variant in ("terms", "batch"):
                e, _ = eng.local_energy(dev(w.logpsi), variant=variant)
                assert np.abs(e.cpu().numpy() - ref).max() <= TOL64
                assert eng.count_pairs(variant) == oracle.find_pairs(w.ham, w.keys)[0].size
        finally:
            eng.set_tuning(0, True, 8)


def test_random_pauli_odd_y(eng):
    """All four letters with odd |Y|: the i^|Y| factor and the ket phase."""
    rng = np.random.default_rng(7)
    ham = jw.random_pauli(10, 300, rng, max_flip=3)
    keys = np.sort(rng.choice(1024, size=400, replace=False)).astype(np.uint64)[:, None]
    keys = keys[rng.permutation(400)]
    lp = rng.normal(size=400) + 1j * rng.uniform(0, 6.28, size=400)
    load(eng, ham, keys)
    ref = oracle.local_energy(ham, keys, lp)
    for variant in ("terms", "batch", "trie"):
        for prec, tol in (("fp64", TOL64), ("fp32c", TOL32)):
            e, _ = eng.local_energy(dev(lp), variant=variant, precision=prec)
            assert np.abs(e.cpu().numpy() - ref).max() <= tol
    ref_p = oracle_pairs(ham, keys)
    for variant in ("batch", "trie"):
        for a, b in zip(gpu_pairs(eng, variant), ref_p):
            np.testing.assert_array_equal(a, b)
    i, j, g = gpu_pairs(eng, "terms")
    h = eng.pair_elements(dev(i, torch.int32), dev(j, torch.int32)).cpu().numpy()
    np.testing.assert_allclose(h, oracle.matrix_elements(ham, keys[i], keys[j]), atol=1e-12)


@pytest.mark.parametrize("partition", [-1, 1])
def test_one_word_wide_keys_mixed_signatures(eng, partition):
    """46 qubits in one key word, so the LoopOverTerms prefilter runs on
    spin-split keys, with keys within three flips of a base key: U has many
    popcount signatures (signature test off) and a small radius around its
    majority key (radius test on).  Pair list bit-exact and E_loc within the
    tolerances against the oracle, unpartitioned and partitioned."""
    rng = np.random.default_rng(31)
    N = 46
    ham = jw.random_pauli(N, 600, rng, max_flip=3)
    base = int(rng.integers(0, 2 ** N))
    rows = set()
    while len(rows) < 2000:
        k = base
        for q in rng.choice(N, size=rng.integers(0, 4), replace=False):
            k ^= 1 << int(q)
        rows.add(k)
    keys = np.array(sorted(rows), dtype=np.uint64)[rng.permutation(len(rows))][:, None]
    lp = rng.normal(scale=0.5, size=keys.shape[0]) + 1j * rng.uniform(0, 6, keys.shape[0])
    eng.set_tuning(partition=partition)
    try:
        load(eng, ham, keys)
        ref_p = oracle_pairs(ham, keys)
        assert ref_p[0].size > 1000
        for a, b in zip(gpu_pairs(eng, "terms"), ref_p):
            np.testing.assert_array_equal(a, b)
        ref = oracle.local_energy(ham, keys, lp)
        for prec, tol in (("fp64", TOL64), ("fp32c", TOL32)):
            e, _ = eng.local_energy(dev(lp), variant="terms", precision=prec)
            assert np.abs(e.cpu().numpy() - ref).max() <= tol * max(1.0, np.abs(ref).max())
    finally:
        eng.set_tuning()


def test_long_group_part_uses_wide_format(eng):
    """A diagonal group of 70 000 Z strings on 20 qubits: its real part is too
    long for the 16-bit run lengths of the narrow hit queue, so the engine
    takes the wide key format; results still match the oracle."""
    rng = np.random.default_rng(11)
    N = 20
    yz_diag = rng.choice(1 << N, size=70000, replace=False).astype(np.uint64)
    off = jw.random_pauli(N, 200, rng, max_flip=4)
    xy = np.concatenate([np.zeros(70000, np.uint64), off.xy[:, 0]])[:, None]
    yz = np.concatenate([yz_diag, off.yz[:, 0]])[:, None]
    coeff = np.concatenate([rng.normal(size=70000) * 1e-3, off.coeff])
    ham = jw.PauliHamiltonian(N, coeff, xy, yz)
    keys = rng.choice(1 << N, size=300, replace=False).astype(np.uint64)[:, None]
    lp = rng.normal(size=300) * 0.2 + 1j * rng.uniform(0, 6.28, size=300)
    load(eng, ham, keys)
    ref = oracle.local_energy(ham, keys, lp)
    for variant in ("terms", "batch", "trie"):
        for prec, tol in (("fp64", TOL64), ("fp32c", TOL32)):
            e, _ = eng.local_energy(dev(lp), variant=variant, precision=prec)
            assert np.abs(e.cpu().numpy() - ref).max() <= tol, (variant, prec)
    ref_p = oracle_pairs(ham, keys)
    for variant in ("terms", "batch", "trie"):
        for a, b in zip(gpu_pairs(eng, variant), ref_p):
            np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("case", ["toy", "odd_y", "small"])
def test_phase_exponents(eng, small_workload, case):
    """Per-(pair, term) phase exponents of MatrixElement, bit for bit against
    the oracle's (themselves pinned by the dense Kronecker build), over the
    engine's own pair list plus uncoupled pairs; H_ij within 1e-12."""
    if case == "toy":
        _, ham, keys, _ = _toy()
    elif case == "odd_y":
        rng = np.random.default_rng(17)
        ham = jw.random_pauli(9, 400, rng, max_flip=3)
        keys = rng.choice(512, size=300, replace=False).astype(np.uint64)[:, None]
    else:
        ham, keys = small_workload.ham, small_workload.keys
    load(eng, ham, keys)
    i, j, _ = gpu_pairs(eng, "terms")
    rng = np.random.default_rng(5)
    extra = rng.integers(0, keys.shape[0], size=(200, 2))     # mostly uncoupled
    i = np.concatenate([i, extra[:, 0]])
    j = np.concatenate([j, extra[:, 1]])
    h, off, k = eng.pair_elements(dev(i, torch.int32), dev(j, torch.int32), phases=True)
    ref_off, ref_k = oracle.phase_exponents(ham, keys[i], keys[j])
    np.testing.assert_array_equal(off.cpu().numpy(), ref_off)
    np.testing.assert_array_equal(k.cpu().numpy(), ref_k)
    np.testing.assert_allclose(h.cpu().numpy(), oracle.matrix_elements(ham, keys[i], keys[j]), atol=1e-12)
    # too small a buffer: ECAPACITY from the deferred check, nothing written
    import paper_2408_07625_amd as pe
    if ref_k.size > 1:
        kk = torch.full((ref_k.size,), 7, dtype=torch.uint8, device="cuda")
        offs = torch.empty(i.size + 1, dtype=torch.int64, device="cuda")
        hh = torch.empty(i.size, dtype=torch.complex128, device="cuda")
        # the index tensors stay referenced until the call has run (a freed
        # temporary's memory can be handed to the next one)
        i_dev, j_dev = dev(i, torch.int32), dev(j, torch.int32)
        rc = eng.lib.eloc_pair_elements(eng.handle, i.size, pe._ptr(i_dev), pe._ptr(j_dev), pe._ptr(hh),
                                        pe._ptr(offs), pe._ptr(kk), ref_k.size - 1)
        assert rc == 0
        with pytest.raises(pe.ElocError) as ex:
            eng.check()
        assert ex.value.status == "ECAPACITY"
        assert bool((kk == 7).all())


def test_deterministic(eng, small_workload):
    w = small_workload
    load(eng, w.ham, w.keys)
    L = dev(w.logpsi)
    for variant in ("terms", "batch", "trie"):
        for prec in ("fp64", "fp32c"):
            a, sa = eng.local_energy(L, variant=variant, precision=prec)
            a = a.clone(); sa = sa.clone()
            b, sb = eng.local_energy(L, variant=variant, precision=prec)
            assert torch.equal(a, b) and torch.equal(sa, sb)


def test_single_determinant(eng):
    """U = {x}: E_loc = H_xx (Slater-Condon closed form checked in the oracle pins)."""
    N = 28
    ham, h, g = jw.random_jw(N, np.random.default_rng(3))
    keys, _ = samples.excitation_batch(N, 14, 1, np.random.default_rng(4))
    load(eng, ham, keys)
    e, st = eng.local_energy(dev(np.array([0.2 - 0.7j])))
    ref = oracle.local_energy(ham, keys, np.array([0.2 - 0.7j]))
    assert abs(e.cpu().numpy()[0] - ref[0]) <= TOL64
    assert abs(st[2].item()) < 1e-18


# ----------------------------------------------------------------------------
def test_errors(eng, small_workload):
    import paper_2408_07625_amd as pe
    w = small_workload
    eng.set_hamiltonian(w.ham.n_qubits, w.ham.coeff, w.ham.xy, w.ham.yz)
    dup = np.concatenate([w.keys[:10], w.keys[3:4]])
    with pytest.raises(pe.ElocError) as ex:
        eng.set_samples(keys_dev(dup))
    assert ex.value.status == "EDUP"
    bad = w.keys[:10].copy()
    bad[5, 0] |= np.uint64(1 << 40)
    with pytest.raises(pe.ElocError) as ex:
        eng.set_samples(keys_dev(bad))
    assert ex.value.status == "EINVAL"
    # the rejected samples stay latched: every synchronising call reports them
    with pytest.raises(pe.ElocError) as ex:
        eng.local_energy(dev(w.logpsi[:10]))
    assert ex.value.status == "EINVAL"
    eng.set_samples(keys_dev(w.keys[:10]))
    negw = np.ones(10)
    negw[2] = -1.0
    with pytest.raises(pe.ElocError) as ex:
        eng.local_energy(dev(w.logpsi[:10]), dev(negw))
    assert ex.value.status == "EINVAL"
    with pytest.raises(pe.ElocError) as ex:
        eng.local_energy(dev(w.logpsi[:10]), dev(np.zeros(10)))
    assert ex.value.status == "EINVAL"
    wide = w.logpsi[:10].copy()
    wide[4] -= 70.0
    with pytest.raises(pe.ElocError) as ex:
        eng.local_energy(dev(wide), precision="fp32c")
    assert ex.value.status == "ERANGE"
    e, _ = eng.local_energy(dev(wide), precision="fp64")     # FP64 takes the wide spread
    ref = oracle.local_energy(w.ham, w.keys[:10], wide)
    assert np.abs(e.cpu().numpy() - ref).max() <= TOL64 * max(1.0, np.abs(ref).max())
    # FP64 up to a spread of 700 (exp of it and of its negative stay normal), not beyond
    wide = w.logpsi[:10].copy()
    wide[4] = wide.real.max() - 690.0 + 1j * wide[4].imag
    e, _ = eng.local_energy(dev(wide), precision="fp64")
    ref = oracle.local_energy(w.ham, w.keys[:10], wide)
    assert np.all(np.abs(e.cpu().numpy() - ref) <= TOL64 * np.maximum(1.0, np.abs(ref)))
    wide[4] -= 20.0
    with pytest.raises(pe.ElocError) as ex:
        eng.local_energy(dev(wide), precision="fp64")
    assert ex.value.status == "ERANGE"
    with pytest.raises(pe.ElocError) as ex:
        eng.pair_elements(dev(np.array([0, 11], dtype=np.int32)), dev(np.array([1, 1], dtype=np.int32)))
    assert ex.value.status == "EINVAL"


# ----------------------------------------------------------------------------
@pytest.mark.parametrize("use_counts", [False, True])
@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_adjoint_small(eng, small_workload, use_counts, precision):
    import paper_2408_07625_amd as pe
    w = small_workload
    load(eng, w.ham, w.keys)
    weights = np.random.default_rng(1).integers(1, 30, size=w.n_unique).astype(float) if use_counts else None
    ref_e = oracle.local_energy(w.ham, w.keys, w.logpsi)
    E, _, _ = oracle.energy(ref_e, w.logpsi, weights)
    for variant in ("terms", "batch", "trie"):
        for ge in (1.0, 1j, 0.3 - 0.4j):
            ref = oracle.adjoint(w.ham, w.keys, w.logpsi, ref_e, ge, weights=weights, energy_value=E)
            L = dev(w.logpsi)
            Wt = None if weights is None else dev(weights)
            e, st = eng.local_energy(L, Wt, variant=variant, precision=precision)
            g = eng.adjoint(L, e, st, ge, Wt, variant=variant, precision=precision).cpu().numpy()
            tol = TOL64 if precision == "fp64" else TOL32
            assert np.abs(g - ref).max() <= tol * max(1.0, np.abs(ref).max())
    # through torch.autograd
    L = dev(w.logpsi).requires_grad_(True)
    Wt = None if weights is None else dev(weights)
    E_t, _, _ = pe.local_energy(eng, L, Wt, "terms", precision)
    E_t.real.backward()
    ref = oracle.adjoint(w.ham, w.keys, w.logpsi, ref_e, 1.0, weights=weights, energy_value=E)
    tol = TOL64 if precision == "fp64" else TOL32
    assert np.abs(L.grad.cpu().numpy() - ref).max() <= tol * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("variant", ["terms", "batch", "trie", "auto"])
@pytest.mark.parametrize("use_counts", [False, True])
def test_stored_pairs(eng, small_workload, variant, use_counts):
    """Forward and adjoint read from the stored pair list: same results as the
    oracle, and the stored list has exactly the oracle's pairs."""
    w = small_workload
    load(eng, w.ham, w.keys)
    weights = np.random.default_rng(2).integers(1, 30, size=w.n_unique).astype(float) if use_counts else None
    n = eng.store_pairs(variant, 1 << 30)
    assert n == oracle_pairs(w.ham, w.keys)[0].size
    ref_e = oracle.local_energy(w.ham, w.keys, w.logpsi)
    E, var, _ = oracle.energy(ref_e, w.logpsi, weights)
    L = dev(w.logpsi)
    Wt = None if weights is None else dev(weights)
    for prec, tol in (("fp64", TOL64), ("fp32c", TOL32)):
        e, st = eng.local_energy(L, Wt, variant="stored", precision=prec)
        assert np.abs(e.cpu().numpy() - ref_e).max() <= tol
        s = st.cpu().numpy()
        assert abs(s[0] - E.real) <= tol and abs(s[2] - var) <= tol * max(1.0, var)
        for ge in (1.0, 0.3 - 0.4j):
            ref = oracle.adjoint(w.ham, w.keys, w.logpsi, ref_e, ge, weights=weights, energy_value=E)
            g = eng.adjoint(L, e, st, ge, Wt, variant="stored", precision=prec).cpu().numpy()
            assert np.abs(g - ref).max() <= tol * max(1.0, np.abs(ref).max())


def test_stored_pairs_budget_and_lifetime(eng, small_workload):
    import paper_2408_07625_amd as pe
    w = small_workload
    load(eng, w.ham, w.keys)
    L = dev(w.logpsi)
    with pytest.raises(pe.ElocError) as ex:
        eng.store_pairs("terms", 1024)
    assert ex.value.status == "ECAPACITY"
    with pytest.raises(pe.ElocError) as ex:
        eng.local_energy(L, None, variant="stored")
    assert ex.value.status == "ESTATE"
    eng.store_pairs("terms", 1 << 30)
    eng.local_energy(L, None, variant="stored")
    eng.set_samples(keys_dev(w.keys))          # new samples invalidate the list
    with pytest.raises(pe.ElocError) as ex:
        eng.local_energy(L, None, variant="stored")
    assert ex.value.status == "ESTATE"
    # through autograd: stored when it fits, recomputed when it does not
    ref_e = oracle.local_energy(w.ham, w.keys, w.logpsi)
    E, _, _ = oracle.energy(ref_e, w.logpsi, None)
    ref = oracle.adjoint(w.ham, w.keys, w.logpsi, ref_e, 1.0, energy_value=E)
    for budget in (1 << 30, 1024):
        Lg = dev(w.logpsi).requires_grad_(True)
        E_t, _, _ = pe.local_energy(eng, Lg, None, "terms", "fp64", store_budget=budget)
        E_t.real.backward()
        assert np.abs(Lg.grad.cpu().numpy() - ref).max() <= TOL64 * max(1.0, np.abs(ref).max())


def test_stored_pairs_wide_sampled(eng):
    """Two-word keys with occurrence counts: stored forward + adjoint on the
    100-qubit workload, sampled rows against the oracle."""
    w = configs.wide()
    load(eng, w.ham, w.keys)
    n = eng.store_pairs("auto", 1 << 36)
    assert n > 0
    L, Wt = dev(w.logpsi), dev(w.weights)
    rows = [(0, 64), ((1 << 18) - 40, 1 << 18)]
    ref = np.concatenate([oracle.local_energy(w.ham, w.keys, w.logpsi, rows=r) for r in rows])
    sel = np.concatenate([np.arange(a, b) for a, b in rows])
    for prec, tol in (("fp64", TOL64), ("fp32c", TOL32)):
        e, st = eng.local_energy(L, Wt, variant="stored", precision=prec)
        assert np.abs(e.cpu().numpy()[sel] - ref).max() <= tol, prec


def test_bloom_filter_opt_in(eng, medium_workload):
    """The opt-in LDS Bloom filter of U (shared by four-wave workgroups) is an
    exact prefilter: same pairs and energies as without it."""
    w = medium_workload
    load(eng, w.ham, w.keys)
    L = dev(w.logpsi)
    rows = (31000, 31400)
    ref = oracle.local_energy(w.ham, w.keys, w.logpsi, rows=rows)
    try:
        eng.set_tuning(0, True, 4, True, 4)
        for prec, tol in (("fp64", TOL64), ("fp32c", TOL32)):
            e, _ = eng.local_energy(L, None, variant="terms", precision=prec)
            assert np.abs(e.cpu().numpy()[rows[0]:rows[1]] - ref).max() <= tol
        assert eng.count_pairs("terms") == 34420502
    finally:
        eng.set_tuning()


# ----------------------------------------------------------------------------
def test_deferred_sample_errors(eng, small_workload):
    """eloc_set_samples is asynchronous: a duplicate key or a bit >= N is
    reported by the next synchronising call, the pair kernels do no work on
    the invalid batch meanwhile, and valid samples afterwards work again."""
    import paper_2408_07625_amd as pe
    w = small_workload
    eng.set_hamiltonian(w.ham.n_qubits, w.ham.coeff, w.ham.xy, w.ham.yz)
    dup = np.concatenate([w.keys[:50], w.keys[7:8]])
    lp = dev(np.concatenate([w.logpsi[:50], w.logpsi[7:8]]))
    eng.set_samples(keys_dev(dup), check=False)
    for variant in ("terms", "batch", "trie"):
        eng.local_energy(lp, variant=variant, check=False)
    with pytest.raises(pe.ElocError) as ex:
        eng.check()
    assert ex.value.status == "EDUP"
    with pytest.raises(pe.ElocError) as ex:
        eng.count_pairs("terms")
    assert ex.value.status == "EDUP"
    bad = w.keys[:50].copy()
    bad[9, 0] |= np.uint64(1 << 20)
    eng.set_samples(keys_dev(bad), check=False)
    with pytest.raises(pe.ElocError) as ex:
        eng.find_pairs("trie")
    assert ex.value.status == "EINVAL"
    eng.set_samples(keys_dev(w.keys[:50]), check=False)
    e, _ = eng.local_energy(dev(w.logpsi[:50]), variant="trie")
    ref = oracle.local_energy(w.ham, w.keys[:50], w.logpsi[:50])
    assert np.abs(e.cpu().numpy() - ref).max() <= TOL64


@pytest.mark.parametrize("shift", [400.0, -400.0])
@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_adjoint_large_log_offset(eng, small_workload, shift, precision):
    """|psi|^2 weights with every Re log psi offset by +-400 (|psi|^2 itself
    over- or underflows): E and the gradient do not change."""
    w = small_workload
    load(eng, w.ham, w.keys)
    lp = w.logpsi + shift
    ref_e = oracle.local_energy(w.ham, w.keys, lp)
    E, _, _ = oracle.energy(ref_e, lp, None)
    ref = oracle.adjoint(w.ham, w.keys, lp, ref_e, 0.3 - 0.4j, energy_value=E)
    L = dev(lp)
    e, st = eng.local_energy(L, None, precision=precision)
    g = eng.adjoint(L, e, st, 0.3 - 0.4j, None, precision=precision).cpu().numpy()
    tol = TOL64 if precision == "fp64" else TOL32
    assert np.all(np.isfinite(g))
    assert np.abs(g - ref).max() <= tol * max(1.0, np.abs(ref).max())


def test_backward_after_state_change_raises(eng, small_workload):
    """A LocalEnergy backward refuses to run when the engine's samples or
    Hamiltonian changed after its forward pass; bad adjoint inputs raise
    before any kernel launch."""
    import paper_2408_07625_amd as pe
    w = small_workload
    load(eng, w.ham, w.keys)
    L = dev(w.logpsi).requires_grad_(True)
    E, e, st = pe.local_energy(eng, L)
    eng.set_samples(keys_dev(w.keys))
    with pytest.raises(RuntimeError, match="changed between the forward"):
        E.real.backward()
    with pytest.raises(ValueError):
        eng.adjoint(dev(w.logpsi[:10]), e, st, 1.0)
    with pytest.raises(ValueError):
        eng.adjoint(dev(w.logpsi), e, st[:3], 1.0)
    with pytest.raises(ValueError):
        eng.adjoint(dev(w.logpsi), e, st, 1.0, weights=dev(np.ones(5)))


# ----------------------------------------------------------------------------
@pytest.mark.parametrize("count", [0, 16, 32])
@pytest.mark.parametrize("wl", ["small", "medium", "odd_y", "two_words"])
def test_partitioned_terms(eng, wl, count, small_workload, medium_workload):
    """LoopOverTerms by U's table partitions (each XCD probing its own
    partitions, one pass after another; on by default only for tables of 8 MB
    and more, forced here, with the automatic count (8 for these tables), 16
    and 32 partitions): forward and adjoint against the oracle in both
    precisions, bitwise reproducible, and the pair list of the variant
    unchanged."""
    if wl == "odd_y":
        rng = np.random.default_rng(21)
        ham = jw.random_pauli(11, 500, rng, max_flip=3)
        keys = rng.choice(2 ** 11, 1500, replace=False).astype(np.uint64)[:, None]
        lp = rng.normal(scale=0.5, size=1500) + 1j * rng.uniform(0, 6, 1500)
    elif wl == "two_words":
        # 70 qubits (two-word keys, membership by fingerprint and key
        # compare): keys within three flips of one base key, so that many
        # pairs couple across both words
        rng = np.random.default_rng(22)
        N = 70
        ham = jw.random_pauli(N, 400, rng, max_flip=2)
        base = np.array([rng.integers(0, 2 ** 62), rng.integers(0, 2 ** (N - 64))], dtype=np.uint64)
        rows = set()
        while len(rows) < 1500:
            k = base.copy()
            for q in rng.choice(N, size=rng.integers(0, 4), replace=False):
                k[q // 64] ^= np.uint64(1) << np.uint64(q % 64)
            rows.add((int(k[0]), int(k[1])))
        keys = np.array(sorted(rows), dtype=np.uint64)[rng.permutation(len(rows))]
        lp = rng.normal(scale=0.5, size=keys.shape[0]) + 1j * rng.uniform(0, 6, keys.shape[0])
    else:
        w = small_workload if wl == "small" else medium_workload
        ham, keys, lp = w.ham, w.keys, w.logpsi
    M = keys.shape[0]
    rows = (0, min(M, 1500))
    eng.set_tuning(partition=1, partition_count=count)
    try:
        load(eng, ham, keys)
        ref = oracle.local_energy(ham, keys, lp, rows=rows)
        L = dev(lp)
        for prec, tol in (("fp64", TOL64), ("fp32c", TOL32)):
            e, st = eng.local_energy(L, variant="terms", precision=prec)
            e1, st1 = e.clone(), st.clone()
            err = np.abs(e.cpu().numpy()[rows[0]:rows[1]] - ref).max()
            print(f"partitioned {wl} {prec}: max |dE_loc| = {err:.2e}")
            assert err <= tol * max(1.0, np.abs(ref).max())
            e2, st2 = eng.local_energy(L, variant="terms", precision=prec)
            assert torch.equal(e1, e2) and torch.equal(st1, st2)
            if M <= 2000:
                E, var, _ = oracle.energy(oracle.local_energy(ham, keys, lp), lp)
                s = st.cpu().numpy()
                assert abs(s[0] - E.real) <= tol and abs(s[2] - var) <= tol * max(1.0, var)
                g = eng.adjoint(L, e, st, 0.3 - 0.4j, None, variant="terms", precision=prec).cpu().numpy()
                gr = oracle.adjoint(ham, keys, lp, oracle.local_energy(ham, keys, lp), 0.3 - 0.4j, energy_value=E)
                assert np.abs(g - gr).max() <= tol * max(1.0, np.abs(gr).max())
        if M <= 2000:
            for a, b in zip(gpu_pairs(eng, "terms"), oracle_pairs(ham, keys)):
                np.testing.assert_array_equal(a, b)
    finally:
        eng.set_tuning()
