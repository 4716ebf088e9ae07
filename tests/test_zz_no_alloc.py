"""The allocation-free forward pass (eloc_local_energy_noalloc) against the
allocating one (eloc_local_energy), through the C ABI: identical outputs bit
for bit (same kernels, same summation order), and within the oracle's
tolerance, on two calls in a row, the second with a smaller input; too large
an input is rejected before any work is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from synth import configs

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "fp32c": 1e-6}


def _call_noalloc(pe, eng, variant, prec, L, Wt, out, stats):
    eng._sync_stream()
    return eng.lib.eloc_local_energy_noalloc(eng.handle, pe.VARIANTS[variant], pe.PRECISIONS[prec], pe._ptr(L),
                                             pe._ptr(Wt), pe._ptr(out), pe._ptr(stats))


def test_noalloc_matches_local_energy():
    import paper_2408_07625_amd as pe
    med, small = configs.medium(), configs.small()
    eng = pe.Engine(0)
    # first the 28-qubit workload (65 536 samples), then the 12-qubit one
    # (1000 samples) on the same device workspace
    for w, use_w in ((med, False), (small, True)):
        M = w.n_unique
        print(f"noalloc: {w.name}, {M} samples", flush=True)
        eng.set_hamiltonian(w.n_qubits, w.ham.coeff, w.ham.xy, w.ham.yz)
        eng.set_samples(torch.from_numpy(w.keys.view(np.int64)).cuda())
        L = torch.from_numpy(w.logpsi).cuda()
        wts = np.arange(1, M + 1, dtype=np.float64) if use_w else None
        Wt = None if wts is None else torch.from_numpy(wts).cuda()
        rows = (0, min(M, 512))
        ref = oracle.local_energy(w.ham, w.keys, w.logpsi, rows=rows)
        E_ref = None
        if M <= 4096:
            full = oracle.local_energy(w.ham, w.keys, w.logpsi)
            E_ref, var_ref, _ = oracle.energy(full, w.logpsi, wts)
        for variant in ("terms", "batch", "auto"):
            for prec in ("fp64", "fp32c"):
                e1, s1 = eng.local_energy(L, Wt, variant, prec)
                e1, s1 = e1.clone(), s1.clone()
                e2 = torch.full((M,), complex("nan"), dtype=torch.complex128, device="cuda")
                s2 = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
                rc = _call_noalloc(pe, eng, variant, prec, L, Wt, e2, s2)
                assert rc == 0, eng.lib.eloc_last_error(eng.handle)
                eng.check()
                assert torch.equal(e1, e2), (w.name, variant, prec)
                assert torch.equal(s1, s2), (w.name, variant, prec)
                err = np.abs(e2.cpu().numpy()[rows[0]:rows[1]] - ref).max()
                assert err <= TOL[prec], (w.name, variant, prec, err)
                if E_ref is not None:
                    s = s2.cpu().numpy()
                    assert abs(s[0] - E_ref.real) <= TOL[prec] and abs(s[2] - var_ref) <= TOL[prec] * max(1, var_ref)
    # the stored pair list is read the same way
    eng.store_pairs("terms")
    e1, s1 = eng.local_energy(L, Wt, "stored", "fp64")
    e1 = e1.clone()
    e2 = torch.empty_like(e1)
    s2 = torch.empty_like(s1)
    assert _call_noalloc(pe, eng, "stored", "fp64", L, Wt, e2, s2) == 0
    eng.check()
    assert torch.equal(e1, e2)
    # LoopOverTrie builds U's sorted copy on first use: refused
    rc = _call_noalloc(pe, eng, "trie", "fp64", L, Wt, e2, s2)
    assert pe.STATUS.get(rc) == "EINVAL"
    eng.close()


def test_noalloc_rejects_oversized_batch():
    """2^20 samples in the FP32C form need more than the fixed workspace:
    ECAPACITY with the size in the message, nothing enqueued."""
    import paper_2408_07625_amd as pe
    from synth import jw
    rng = np.random.default_rng(11)
    ham = jw.random_pauli(40, 200, rng, max_flip=2)
    M = 1 << 20
    keys = np.unique(rng.integers(0, 1 << 40, size=M + M // 8, dtype=np.int64))[:M]
    assert keys.size == M
    eng = pe.Engine(0)
    eng.set_hamiltonian(40, ham.coeff, ham.xy, ham.yz)
    eng.set_samples(torch.from_numpy(keys.reshape(M, 1)).cuda())
    L = torch.zeros(M, dtype=torch.complex128, device="cuda")
    out = torch.full((M,), 7.0 + 0j, dtype=torch.complex128, device="cuda")
    stats = torch.zeros(4, dtype=torch.float64, device="cuda")
    rc = _call_noalloc(pe, eng, "terms", "fp32c", L, None, out, stats)
    assert pe.STATUS.get(rc) == "ECAPACITY"
    assert b"fixed workspace" in eng.lib.eloc_last_error(eng.handle)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    eng.close()
