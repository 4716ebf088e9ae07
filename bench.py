"""Throughput of the sample-aware local energy on one MI355X.

A step is one pass of the hot path over one batch: prepare U (copy, hash
table, duplicate and bit checks), then FindCoupledPairs + MatrixElement +
ratio accumulation (one fused kernel), the per-row combination and the
weighted energy / variance reductions.  Hamiltonian ingest is done once,
before timing, as the paper precomputes it.

Workload: 28 qubits, 14 electrons, 65 536 unique determinants (HF plus
rank <= 4 excitations), JW Hamiltonian from seeded random integrals; inputs
are resident in device memory before timing starts.

Prints one JSON line.  value = coupled pairs/s of the compensated-FP32 form;
the plain FP64 form is reported beside it.  The "batched" object times the
64-problem batched launch (qubit counts 16..40, unique batches 10^3..10^5,
one persistent launch replayed from a HIP graph, autotuned schedule)
against the same problems run as 64 sequential single launches.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

PROFILES = ROOT / "profiles"
PAIR_SOURCES = [ROOT / "paper_2408_07625_amd" / "csrc" / f for f in ("pairs.hip", "device.h", "internal.h")]


def pair_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for p in PAIR_SOURCES:
        h.update(p.read_bytes())
    return h.hexdigest()[:16]


def measured_traffic(name: str):
    """HBM bytes per launch of the pair kernel from a committed counter
    summary, if it was taken on the current kernel source; else None."""
    path = PROFILES / name
    if not path.exists():
        return None
    fields = {}
    for line in path.read_text().splitlines():
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("source_hash") != pair_source_hash():
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# Algorithmic lane-op counts per unit of work of the fused pair kernel (W
# 64-bit words per key); see the design notes for the derivation.
def ops_per_candidate(W):
    return 2 * W + 3          # x ^ XY (2W), hash combine (2), slot index (1)


def ops_per_term(W):
    return 4 * W + 3          # AND + popcount of ket & YZ (4W), parity select (2), add (1)


OPS_PER_PAIR = 4              # complex multiply-accumulate: 4 FMAs
PEAK_LANE_OPS = 256 * 64 * 2.4e9   # CUs x lanes/clock x clock: 3.93e13 lane-ops/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="medium")
    ap.add_argument("--variant", default="terms")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", action="store_true", help="time only the headline variant")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-launch measurement")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the forward + adjoint measurement")
    ap.add_argument("--calibrate-mib", type=int, default=0,
                    help="also run a plain elementwise copy of this many MiB (reads and writes it once), "
                         "the reference kernel for scaling hardware byte counters")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this engine runs on one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2408_07625_amd as pe
    from synth import configs

    w = configs.by_name(args.workload)
    M, N, W = w.n_unique, w.n_qubits, w.ham.n_words
    eng = pe.Engine(0)
    eng.set_hamiltonian(N, w.ham.coeff, w.ham.xy, w.ham.yz)
    info = eng.info()
    keys = torch.from_numpy(w.keys.view(np.int64)).cuda()
    L = torch.from_numpy(w.logpsi).cuda()
    Wt = None if w.weights is None else torch.from_numpy(w.weights).cuda()
    out = torch.empty(M, dtype=torch.complex128, device="cuda")
    stats = torch.empty(4, dtype=torch.float64, device="cuda")
    print(f"# workload {w.name}: N={N} M={M} terms={info['n_terms']} groups={info['n_groups']}",
          file=sys.stderr, flush=True)

    def step(prec):
        eng.set_samples(keys, check=False)
        eng.local_energy(L, Wt, args.variant, prec, out=out, stats=stats, check=False)

    results = {}
    for prec in ("fp64", "fp32c"):
        for _ in range(args.warmup):
            step(prec)
        eng.check()
        torch.cuda.synchronize()
        eng.profile(True)
        eng.profile_read()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(args.steps):
            step(prec)
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        eng.check()
        prof = eng.profile_read()
        eng.profile(False)
        ms = e0.elapsed_time(e1) / args.steps
        results[prec] = {"ms_per_step": ms, "wall_ms_per_step": 1e3 * wall / args.steps, "stages": prof,
                         "eloc": out.cpu().numpy().copy(), "stats": stats.cpu().numpy().copy()}
        print(f"# {prec}: {ms:.3f} ms/step  stages(ms/launch): " +
              ", ".join(f"{k}={v[0] / max(v[1], 1):.3f}" for k, v in prof.items() if v[1]),
              file=sys.stderr, flush=True)

    # the other FindCoupledPairs variants, same workload and protocol
    variants = {}
    for var in ("terms", "batch", "trie"):
        if var == args.variant or args.only:
            continue
        for prec in ("fp64", "fp32c"):
            for _ in range(args.warmup):
                eng.set_samples(keys, check=False)
                eng.local_energy(L, Wt, var, prec, out=out, stats=stats, check=False)
            eng.check()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.steps):
                eng.set_samples(keys, check=False)
                eng.local_energy(L, Wt, var, prec, out=out, stats=stats, check=False)
            e1.record()
            torch.cuda.synchronize()
            eng.check()
            variants.setdefault(var, {})[prec] = e0.elapsed_time(e1) / args.steps
        print(f"# variant {var}: " + ", ".join(f"{p}={v:.3f} ms/step" for p, v in variants[var].items()),
              file=sys.stderr, flush=True)

    # work counts (outside the timed region)
    n_pairs = eng.count_pairs(args.variant)
    _, _, gids = eng.find_pairs(args.variant)
    # terms per group, groups numbered in first-appearance order of their XY mask
    _, first, inv, cnt = np.unique(w.ham.xy, axis=0, return_index=True, return_inverse=True,
                                   return_counts=True)
    rank = np.empty(first.size, dtype=np.int64)
    rank[np.argsort(first)] = np.arange(first.size)
    sizes = np.zeros(first.size, dtype=np.int64)
    sizes[rank] = cnt
    term_evals = int(sizes[gids.cpu().numpy()].sum())
    candidates = M * info["n_groups"] if args.variant == "terms" else M * M

    headline = results["fp32c"]
    pairs_s = n_pairs / (headline["ms_per_step"] * 1e-3)
    samples_s = M / (headline["ms_per_step"] * 1e-3)
    fp64 = results["fp64"]

    # roofline of the dominant kernel (fused pair kernel), ALU bound
    pair_ms, pair_n = headline["stages"]["pairs"]
    pair_avg_s = pair_ms / max(pair_n, 1) * 1e-3
    ops = candidates * ops_per_candidate(W) + term_evals * ops_per_term(W) + n_pairs * OPS_PER_PAIR
    achieved = ops / pair_avg_s
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12, "unit": "Tlane-op/s",
            "frac": achieved / PEAK_LANE_OPS,
            "traffic": measured_traffic(f"k_pairs_{w.name}_{args.variant}_fp32c_traffic.md"),
            "kernel": "k_pairs (fused FindCoupledPairs + MatrixElement + accumulation)",
            "kernel_ms": pair_avg_s * 1e3,
            "ops_per_launch": ops}

    rec = {
        "metric": "coupled pairs/sec + E_loc^var samples/sec vs plain FP64 at |dE|<=1e-6 Ha",
        "value": pairs_s, "unit": "coupled pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": headline["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32c", "data": "synthetic",
        "config": {"workload": f"{w.name}: {N} qubits, {w.n_electrons} electrons, {M} unique determinants, "
                               f"{info['n_terms']} Pauli terms in {info['n_groups']} XY groups",
                   "variant": args.variant, "global_batch": M},
        "samples_per_s": samples_s,
        "coupled_pairs": n_pairs, "candidates": candidates, "term_evaluations": term_evals,
        "fp64": {"pairs_per_s": n_pairs / (fp64["ms_per_step"] * 1e-3),
                 "samples_per_s": M / (fp64["ms_per_step"] * 1e-3), "ms_per_step": fp64["ms_per_step"]},
        "fp32c_over_fp64": fp64["ms_per_step"] / headline["ms_per_step"],
        "stage_ms": {p: {k: v[0] / max(v[1], 1) for k, v in results[p]["stages"].items() if v[1]}
                     for p in results},
        "roofline": roof,
        "other_variants_ms_per_step": variants,
    }

    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        ref = oracle.local_energy(w.ham, w.keys, w.logpsi)
        cpu_s = time.perf_counter() - t0
        E_ref, var_ref, _ = oracle.energy(ref, w.logpsi, w.weights)
        rec["accuracy"] = {
            p: {"max_abs_dE_loc": float(np.abs(results[p]["eloc"] - ref).max()),
                "abs_dE": float(abs(results[p]["stats"][0] + 1j * results[p]["stats"][1] - E_ref)),
                "abs_dVar": float(abs(results[p]["stats"][2] - var_ref))} for p in results}
        rec["energy"] = {"E": E_ref.real, "Var": var_ref}
        if not args.no_cpu_baseline:
            rec["cpu_baseline"] = {"value": n_pairs / cpu_s, "unit": "coupled pairs/s",
                                   "cores": oracle.max_threads(), "kind": "oracle",
                                   "sample": f"all {M} rows of the workload, one forward pass "
                                             f"({cpu_s:.2f} s wall)",
                                   "samples_per_s": M / cpu_s}
    if not args.no_batched:
        rec["batched"] = bench_batched(args)
    if not args.no_adjoint:
        rec["adjoint"] = bench_adjoint(args)
    if args.calibrate_mib:
        n = args.calibrate_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        rec["calibration_copy_bytes"] = 2 * n * 8
    print(json.dumps(rec))
    eng.close()


def bench_adjoint(args):
    """Forward and adjoint (dE/dlog psi) on the 100-qubit workload (two-word
    keys, 2^18 samples, occurrence counts), pairs recomputed by the adjoint."""
    import numpy as np
    import torch

    import paper_2408_07625_amd as pe
    from synth import configs

    t0 = time.perf_counter()
    w = configs.wide()
    eng = pe.Engine(0)
    eng.set_hamiltonian(w.n_qubits, w.ham.coeff, w.ham.xy, w.ham.yz)
    info = eng.info()
    keys = torch.from_numpy(w.keys.view(np.int64)).cuda()
    L = torch.from_numpy(w.logpsi).cuda()
    Wt = torch.from_numpy(w.weights).cuda()
    eng.set_samples(keys)
    M = w.n_unique
    out = torch.empty(M, dtype=torch.complex128, device="cuda")
    stats = torch.empty(4, dtype=torch.float64, device="cuda")
    grad = torch.empty(M, dtype=torch.complex128, device="cuda")
    variant = "batch" if M <= info["n_groups"] else "terms"
    print(f"# adjoint workload: {w.n_qubits} qubits, {M} samples, {info['n_terms']} terms, "
          f"{info['n_groups']} groups, variant {variant} (set up in {time.perf_counter() - t0:.1f} s)",
          file=sys.stderr, flush=True)
    steps = max(2, args.steps // 5)

    def timed(fn):
        for _ in range(max(1, args.warmup)):
            fn()
        eng.check()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        eng.check()
        return e0.elapsed_time(e1) / steps

    res = {"workload": f"wide: {w.n_qubits} qubits (two-word keys), {w.n_electrons} electrons, {M} unique "
                       f"determinants, {info['n_terms']} Pauli terms in {info['n_groups']} XY groups, "
                       f"occurrence-count weights", "variant": variant, "steps": steps}
    for prec in ("fp64", "fp32c"):
        fwd = timed(lambda: eng.local_energy(L, Wt, variant, prec, out=out, stats=stats, check=False))
        adj = timed(lambda: eng.adjoint(L, out, stats, 1.0 + 0.0j, Wt, variant, prec, out=grad, check=False))
        res[prec] = {"forward_ms": fwd, "adjoint_ms": adj}
        print(f"# adjoint {prec}: forward {fwd:.3f} ms, adjoint {adj:.3f} ms", file=sys.stderr, flush=True)
    n_pairs = eng.count_pairs(variant)
    res["coupled_pairs"] = n_pairs
    for prec in ("fp64", "fp32c"):
        res[prec]["pairs_per_s_forward_plus_adjoint"] = 2 * n_pairs / (
            (res[prec]["forward_ms"] + res[prec]["adjoint_ms"]) * 1e-3)
    eng.close()
    return res


def bench_batched(args):
    """The batched launch over 64 problems against 64 sequential launches."""
    import numpy as np
    import torch

    import paper_2408_07625_amd as pe
    from synth import configs

    t0 = time.perf_counter()
    ws = configs.batched()
    probs = [{"n_qubits": w.n_qubits, "coeff": w.ham.coeff, "xy": w.ham.xy, "yz": w.ham.yz,
              "keys": torch.from_numpy(w.keys.view(np.int64)).cuda(), "logpsi": torch.from_numpy(w.logpsi).cuda()}
             for w in ws]
    b = pe.Batch(probs)
    S = sum(w.n_unique for w in ws)
    print(f"# batched: {len(ws)} problems, {S} samples, {sum(w.ham.n_terms for w in ws)} terms "
          f"(set up in {time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    schedule, _ = b.tune("fp32c")
    tune_s = time.perf_counter() - t0
    print(f"# batched: tuned in {tune_s:.1f} s: {schedule}", file=sys.stderr, flush=True)

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    out = {"workload": f"{len(ws)} problems: {min(w.n_qubits for w in ws)}..{max(w.n_qubits for w in ws)} qubits, "
                       f"{S} unique samples in all ({min(w.n_unique for w in ws)}..{max(w.n_unique for w in ws)} "
                       f"per problem), |psi|^2 weights",
           "schedule": schedule, "tune_s": tune_s}
    for prec in ("fp32c", "fp64"):
        b.set_graph(True)
        ms = timed(lambda: b.run(prec, check=False), args.steps)
        b.check()
        pairs = int(b.pair_counts().sum())
        b.set_graph(False)
        ms_eager = timed(lambda: b.run(prec, check=False), args.steps)
        b.check()
        b.set_graph(True)
        out[prec] = {"ms_per_step": ms, "pairs_per_s": pairs / (ms * 1e-3), "samples_per_s": S / (ms * 1e-3),
                     "eager_ms_per_step": ms_eager}
        out["coupled_pairs"] = pairs
        print(f"# batched {prec}: graph {ms:.3f} ms, eager {ms_eager:.3f} ms, {pairs} pairs",
              file=sys.stderr, flush=True)
    # the same problems one by one: one context each (Hamiltonian ingested
    # once), each step sets the samples and runs the forward pass
    engines = []
    for k, w in enumerate(ws):
        e = pe.Engine(0)
        e.set_hamiltonian(w.n_qubits, w.ham.coeff, w.ham.xy, w.ham.yz)
        info = b.problem_info(k)
        engines.append((e, info["variant"], probs[k]["keys"], probs[k]["logpsi"],
                        torch.empty(w.n_unique, dtype=torch.complex128, device="cuda"),
                        torch.empty(4, dtype=torch.float64, device="cuda")))

    def sequential(prec):
        for e, var, keys, L, o, s in engines:
            e.set_samples(keys, check=False)
            e.local_energy(L, None, var, prec, out=o, stats=s, check=False)

    for prec in ("fp32c", "fp64"):
        ms = timed(lambda: sequential(prec), max(1, args.steps // 4))
        out[prec]["sequential_ms_per_step"] = ms
        out[prec]["speedup_vs_sequential"] = ms / out[prec]["ms_per_step"]
        print(f"# sequential {prec}: {ms:.3f} ms", file=sys.stderr, flush=True)
    out["fp32c_over_fp64"] = out["fp64"]["ms_per_step"] / out["fp32c"]["ms_per_step"]
    for e, *_ in engines:
        e.close()
    b.close()
    return out


if __name__ == "__main__":
    main()
