"""Batched launch (eloc_batch_*) against the oracle, per problem.

Every problem of a batch must give what the oracle gives for it alone:
E_loc^var per sample and the weighted statistics within the tolerances of
the single-problem tests, and exactly the oracle's number of coupled pairs.
With the same chunking and rows per wave, E_loc must equal the
single-problem launch bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from synth import configs, jw

pytestmark = pytest.mark.gpu

TOL64 = 1e-9
TOL32 = 1e-6


@pytest.fixture(scope="module")
def pe():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2408_07625_amd as pe
    return pe


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def as_problem(w, weights=None):
    return {"n_qubits": w.n_qubits, "coeff": w.ham.coeff, "xy": w.ham.xy, "yz": w.ham.yz,
            "keys": dev(w.keys.view(np.int64)), "logpsi": dev(w.logpsi),
            "weights": None if weights is None else dev(weights)}


def odd_y_problem():
    """A 70-qubit random Pauli Hamiltonian (two words per key, odd |Y| terms,
    plus Z-only diagonal terms) with keys that differ from a base state by
    up to two of its XY masks: exercises word padding and the i^|Y| phase."""
    rng = jw.rng_for(41, 0)
    N = 70
    ham = jw.random_pauli(N, 300, rng, max_flip=3)
    zs = jw.random_pauli(N, 20, rng, max_flip=0)
    ham = jw.PauliHamiltonian(N, np.concatenate([ham.coeff, zs.coeff]), np.concatenate([ham.xy, zs.xy]),
                              np.concatenate([ham.yz, zs.yz]))
    base = np.array([rng.integers(0, 1 << 62), rng.integers(0, 1 << 6)], dtype=np.uint64)
    seen, rows = set(), []
    while len(rows) < 400:
        x = base.copy()
        for t_ in rng.choice(300, size=rng.integers(0, 3), replace=False):
            x ^= ham.xy[t_]
        if tuple(x.tolist()) not in seen:
            seen.add(tuple(x.tolist()))
            rows.append(x)
    k = np.array(rows, dtype=np.uint64)
    lp = rng.normal(-1.0, 0.5, size=k.shape[0]) + 1j * rng.uniform(0, 2 * np.pi, size=k.shape[0])
    return configs.Workload("odd_y70", 0, ham, k, lp, None)


@pytest.fixture(scope="module")
def small_batch():
    ws = configs.batched(n_problems=10, n_min=8, n_max=20, u_min=20, u_max=3000, cfg=40)
    ws.append(odd_y_problem())
    one = configs.batched(n_problems=1, n_min=12, n_max=12, u_min=1, u_max=1, cfg=41)[0]
    ws.append(one)     # a single sample
    return ws


@pytest.fixture(scope="module")
def reference(small_batch):
    out = []
    for w in small_batch:
        e, npairs = oracle.local_energy(w.ham, w.keys, w.logpsi, with_pairs=True)
        E, var, tot = oracle.energy(e, w.logpsi, w.weights)
        out.append((e, int(npairs.sum()), E, var, tot))
    return out


def check_against(batch, ws, ref, tol):
    counts = batch.pair_counts()
    for k, (w, (e, npairs, E, var, tot)) in enumerate(zip(ws, ref)):
        got = batch.eloc[k].cpu().numpy()
        err = np.abs(got - e).max()
        assert err <= tol, (k, w.name, err)
        s = batch.stats[k].cpu().numpy()
        assert abs(s[0] - E.real) <= tol and abs(s[1] - E.imag) <= tol, (k, s, E)
        assert abs(s[2] - var) <= tol * max(1.0, var), (k, s[2], var)
        np.testing.assert_allclose(s[3], tot, rtol=1e-12)
        assert counts[k] == npairs, (k, counts[k], npairs)


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32c", TOL32)])
def test_batch_matches_oracle(pe, small_batch, reference, precision, tol):
    b = pe.Batch([as_problem(w) for w in small_batch])
    b.run(precision)
    check_against(b, small_batch, reference, tol)
    # the graph replays the current inputs: change them in place and run again
    ws2 = []
    for k, w in enumerate(small_batch):
        lp = w.logpsi + 0.1 * np.cos(np.arange(w.n_unique)) + 0.05j
        b.inputs[k]["logpsi"].copy_(dev(lp))
        ws2.append(configs.Workload(w.name, w.n_electrons, w.ham, w.keys, lp, None))
    ref2 = []
    for w in ws2:
        e, npairs = oracle.local_energy(w.ham, w.keys, w.logpsi, with_pairs=True)
        E, var, tot = oracle.energy(e, w.logpsi, None)
        ref2.append((e, int(npairs.sum()), E, var, tot))
    for _ in range(3):
        b.run(precision)
        check_against(b, ws2, ref2, tol)


@pytest.mark.parametrize("sched", [dict(rows_per_wave=4, item_candidates=1 << 12, batch_ratio=0.0),
                                   dict(rows_per_wave=8, item_candidates=1 << 20, batch_ratio=1e9, order=1),
                                   dict(rows_per_wave=4, item_candidates=64, batch_ratio=1.0, blocks_per_cu=1)])
@pytest.mark.parametrize("words", ["mixed", "one"])
def test_schedules_agree(pe, small_batch, reference, sched, words):
    # "one": only the problems of one-word keys, so the batch runs W = 1
    n = len(small_batch) if words == "mixed" else 10
    ws, ref = small_batch[:n], reference[:n]
    b = pe.Batch([as_problem(w) for w in ws])
    b.set_schedule(**sched)
    for precision, tol in (("fp64", TOL64), ("fp32c", TOL32)):
        b.run(precision)
        check_against(b, ws, ref, tol)


def test_graph_and_eager_identical(pe, small_batch):
    b = pe.Batch([as_problem(w) for w in small_batch])
    for precision in ("fp64", "fp32c"):
        b.set_graph(True)
        b.run(precision)
        g = [e.cpu().numpy().copy() for e in b.eloc]
        b.set_graph(False)
        b.run(precision)
        for k, e in enumerate(b.eloc):
            np.testing.assert_array_equal(e.cpu().numpy(), g[k])


def test_bitwise_equal_to_single_launch(pe, small_batch):
    """Same chunking and rows per wave: identical rows, bit for bit."""
    b = pe.Batch([as_problem(w) for w in small_batch])
    eng = pe.Engine(0)
    for rows in (4, 8):
        b.set_schedule(rows_per_wave=rows, item_candidates=1 << 13, batch_ratio=1.0)
        for precision in ("fp64", "fp32c"):
            b.run(precision)
            for k, w in enumerate(small_batch):
                info = b.problem_info(k)
                eng.set_hamiltonian(w.n_qubits, w.ham.coeff, w.ham.xy, w.ham.yz)
                eng.set_samples(dev(w.keys.view(np.int64)))
                eng.set_tuning(chunks=info["chunks"], sig_filter=True, rows_per_wave=rows)
                e, _ = eng.local_energy(dev(w.logpsi), variant=info["variant"], precision=precision)
                np.testing.assert_array_equal(b.eloc[k].cpu().numpy(), e.cpu().numpy(), err_msg=f"{k} {info}")


def test_weights_and_errors(pe, small_batch):
    ws = small_batch[:3]
    rng = np.random.default_rng(5)
    weights = [rng.integers(1, 20, size=w.n_unique).astype(np.float64) for w in ws]
    probs = [as_problem(w, wt) for w, wt in zip(ws, weights)]
    b = pe.Batch(probs)
    b.run("fp64")
    for k, w in enumerate(ws):
        e = oracle.local_energy(w.ham, w.keys, w.logpsi)
        E, var, tot = oracle.energy(e, w.logpsi, weights[k])
        s = b.stats[k].cpu().numpy()
        assert abs(s[0] - E.real) <= TOL64 and abs(s[2] - var) <= TOL64 * max(1, var)
        assert s[3] == tot
    # a duplicate key in problem 1
    keys1 = b.inputs[1]["keys"]
    saved = keys1.clone()
    keys1[1] = keys1[0]
    with pytest.raises(pe.ElocError) as ex:
        b.run("fp64")
    assert ex.value.status == "EDUP" and ex.value.problem == 1
    keys1.copy_(saved)
    # a bit at or above n_qubits in problem 2
    keys2 = b.inputs[2]["keys"]
    saved = keys2.clone()
    keys2[0, 0] = saved[0, 0] | (1 << ws[2].n_qubits)
    with pytest.raises(pe.ElocError) as ex:
        b.run("fp64")
    assert ex.value.status == "EINVAL" and ex.value.problem == 2
    keys2.copy_(saved)
    # negative weight in problem 0
    w0 = b.inputs[0]["weights"]
    w0[0] = -1.0
    with pytest.raises(pe.ElocError) as ex:
        b.run("fp64")
    assert ex.value.status == "EINVAL" and ex.value.problem == 0
    w0[0] = 1.0
    # FP32C range: one log-amplitude far below the rest
    lp0 = b.inputs[0]["logpsi"]
    lp0[0] = lp0[0] - 70.0
    with pytest.raises(pe.ElocError) as ex:
        b.run("fp32c")
    assert ex.value.status == "ERANGE" and ex.value.problem == 0
    lp0[0] = lp0[0] + 70.0
    b.run("fp64")


def long_part_problem():
    """20 qubits, a diagonal group of 70 000 Z strings (longer than the narrow
    hit queue's 16-bit run lengths) plus random off-diagonal terms."""
    rng = np.random.default_rng(12)
    N = 20
    off = jw.random_pauli(N, 200, rng, max_flip=4)
    xy = np.concatenate([np.zeros(70000, np.uint64), off.xy[:, 0]])[:, None]
    yz = np.concatenate([rng.choice(1 << N, size=70000, replace=False).astype(np.uint64), off.yz[:, 0]])[:, None]
    ham = jw.PauliHamiltonian(N, np.concatenate([rng.normal(size=70000) * 1e-3, off.coeff]), xy, yz)
    keys = rng.choice(1 << N, size=300, replace=False).astype(np.uint64)[:, None]
    lp = rng.normal(size=300) * 0.2 + 1j * rng.uniform(0, 6.28, size=300)
    return configs.Workload("long_part20", 0, ham, keys, lp, None)


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32c", TOL32)])
def test_long_group_part_in_batch(pe, small_batch, reference, precision, tol):
    """A narrow batch with one problem whose group part is too long for the
    narrow hit queue runs in the wide key format, and still matches."""
    ws = [w for w in small_batch if w.n_qubits <= 32] + [long_part_problem()]
    ref = [r for w, r in zip(small_batch, reference) if w.n_qubits <= 32]
    w = ws[-1]
    e, npairs = oracle.local_energy(w.ham, w.keys, w.logpsi, with_pairs=True)
    E, var, tot = oracle.energy(e, w.logpsi, None)
    ref.append((e, int(npairs.sum()), E, var, tot))
    b = pe.Batch([as_problem(w) for w in ws])
    b.run(precision)
    check_against(b, ws, ref, tol)


def test_tune_and_cache(pe, small_batch, reference, tmp_path):
    b = pe.Batch([as_problem(w) for w in small_batch])
    cache = tmp_path / "schedule.txt"
    s1, hit1 = b.tune("fp32c", cache)
    assert not hit1 and cache.exists()
    b.run("fp32c")
    check_against(b, small_batch, reference, TOL32)
    b2 = pe.Batch([as_problem(w) for w in small_batch])
    s2, hit2 = b2.tune("fp32c", cache)
    assert hit2 and s2 == s1


def test_full_size_batch_sampled():
    """The 64-problem workload at full size: pair counts of every problem
    against the single-problem launch, and sampled rows of a few problems
    against the oracle."""
    import paper_2408_07625_amd as pe
    ws = configs.batched()
    b = pe.Batch([as_problem(w) for w in ws])
    b.tune("fp32c")
    for precision, tol in (("fp64", TOL64), ("fp32c", TOL32)):
        b.run(precision)
        counts = b.pair_counts()
        for k in range(0, len(ws), 9):
            w = ws[k]
            rows = (0, min(w.n_unique, 150))
            e, npairs = oracle.local_energy(w.ham, w.keys, w.logpsi, rows=rows, with_pairs=True)
            got = b.eloc[k].cpu().numpy()[rows[0]:rows[1]]
            assert np.abs(got - e).max() <= tol, (k, precision)
        if precision == "fp64":
            eng = pe.Engine(0)
            for k in range(0, len(ws), 5):
                w = ws[k]
                eng.set_hamiltonian(w.n_qubits, w.ham.coeff, w.ham.xy, w.ham.yz)
                eng.set_samples(dev(w.keys.view(np.int64)))
                assert eng.count_pairs("terms") == counts[k], k
