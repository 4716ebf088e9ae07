"""Throughput of the sample-aware local energy on one MI355X.

A step is one pass of the hot path over one batch: prepare U (copy, hash
table, duplicate and bit checks), then FindCoupledPairs + MatrixElement +
ratio accumulation (one fused kernel), the per-row combination and the
weighted energy / variance reductions.  Hamiltonian ingest is done once,
before timing, as the paper precomputes it.

Headline workload (default): 52 qubits, 20 electrons, 2^20 unique
determinants (HF plus rank <= 4 excitations), JW Hamiltonian from seeded
random integrals (669 579 Pauli terms); inputs are resident in device memory
before timing starts.  All three FindCoupledPairs variants are timed in both
precisions, with the per-stage breakdown.

Prints one JSON line.  value = coupled pairs/s of the compensated-FP32 form
of the headline variant; the plain FP64 form is reported beside it.  Extra
objects: "medium" (28 qubits, 65 536 samples), "batched" (64 problems in one
persistent launch replayed from a HIP graph, against 64 sequential
launches), "adjoint" (100 qubits, forward + dE/dlog psi).
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
GOLDEN = ROOT / "tests" / "golden"
PAIR_SOURCES = [ROOT / "paper_2408_07625_amd" / "csrc" / f for f in ("pairs.hip", "device.h", "internal.h")]

PEAK_LANE_OPS = 256 * 64 * 2.4e9   # CUs x lanes x clock: one wave instruction per CU per clock
PEAK_HBM = 8.0e12                  # bytes/s


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


# Algorithmic lane-operations per unit of work (W 64-bit words per key):
#  LoopOverTerms candidate: x ^ XY (2W int32 ops) + one hash probe (~10);
#  LoopOverBatch candidate: x ^ x' (2W), popcount (2W), compare + ballot (2);
#  term evaluation: AND + popcount of ket & YZ, parity select, add (~12);
#  coupled pair: one complex multiply-accumulate, 4 FP64 FMAs or about 30
#  FP32 operations in the compensated form (TwoProduct x4 + TwoSum x2).
#  LoopOverTrie node-pair visit: masked XOR of row, U and XY keys over the
#  bit run (4W), branch-bit compare, child selection and push (~10).
def ops_per_candidate(variant: str, W: int) -> int:
    if variant == "terms":
        return 2 * W + 10
    if variant == "trie":
        return 4 * W + 10
    return 4 * W + 2


OPS_PER_TERM = 12
OPS_PER_PAIR = {"fp64": 4, "fp32c": 30}


def cpu_model() -> str:
    try:
        for line in Path("/proc/cpuinfo").read_text().splitlines():
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large")
    ap.add_argument("--variant", default="terms", help="headline FindCoupledPairs variant")
    ap.add_argument("--other-steps", type=int, default=5, help="timed steps of the other variants (at most --steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", action="store_true", help="time only the headline variant")
    ap.add_argument("--no-medium", action="store_true", help="skip the 28-qubit object")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-launch measurement")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the forward + adjoint measurement")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the conventional local energy, SR and sampler measurements")
    ap.add_argument("--partition", type=int, default=0,
                    help="LoopOverTerms by U's table partitions: 0 automatic, 1 on, -1 off")
    ap.add_argument("--partition-count", type=int, default=0, help="table partitions: 8, 16, 32 (0 automatic)")
    ap.add_argument("--calibrate-mib", type=int, default=0,
                    help="also run a plain elementwise copy of this many MiB (reads and writes it once), "
                         "the reference kernel for scaling hardware byte counters")
    return ap.parse_args()


def group_sizes_by_id(ham):
    """Terms per XY group, groups numbered in first-appearance order."""
    import numpy as np
    _, first, cnt = np.unique(ham.xy, axis=0, return_index=True, return_counts=True)
    rank = np.empty(first.size, dtype=np.int64)
    rank[np.argsort(first)] = np.arange(first.size)
    sizes = np.zeros(first.size, dtype=np.int64)
    sizes[rank] = cnt
    return sizes


def term_evaluations(eng, variant, sizes):
    """Sum over the coupled pairs of their group's term count (on the GPU)."""
    import torch
    _, _, g = eng.find_pairs(variant)
    sz = torch.from_numpy(sizes).cuda()
    total = 0
    step = 1 << 27
    for a in range(0, g.numel(), step):
        total += int(sz[g[a:a + step].long()].sum().item())
    del g
    torch.cuda.empty_cache()
    return total


def time_steps(eng, step, steps, warmup):
    """W warm-up steps, then K timed steps between synchronisations, HIP
    events on the engine's stream around each stage (eloc_profile_*)."""
    import torch
    for _ in range(warmup):
        step()
    eng.check()
    torch.cuda.synchronize()
    eng.profile(True)
    eng.profile_read()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    eng.check()
    prof = eng.profile_read()
    eng.profile(False)
    return e0.elapsed_time(e1) / steps, prof


def roofline(variant, prec, W, M, n_terms, n_groups, cand, term_evals, n_pairs, kernel_s, traffic):
    ops = cand * ops_per_candidate(variant, W) + term_evals * OPS_PER_TERM + n_pairs * OPS_PER_PAIR[prec]
    # compulsory bytes of one launch: keys, amplitudes in, row sums out,
    # the term and group records of the Hamiltonian
    compulsory = M * (8 * W + 16 + 16) + n_terms * (8 * W + 8) + n_groups * (8 * W + 8)
    achieved = ops / kernel_s
    r = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12, "unit": "Tlane-op/s",
         "frac": achieved / PEAK_LANE_OPS, "traffic": traffic,
         "kernel": f"k_pairs {variant} {prec} (fused FindCoupledPairs + MatrixElement + accumulation)",
         "kernel_ms": kernel_s * 1e3, "ops_per_launch": ops,
         "hbm": {"compulsory_bytes": compulsory, "compulsory_frac": compulsory / kernel_s / PEAK_HBM,
                 "counter_bytes": traffic,
                 "counter_frac": None if traffic is None else traffic / kernel_s / PEAK_HBM}}
    return r


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

    t0 = time.perf_counter()
    w = configs.by_name(args.workload)
    M, N, W = w.n_unique, w.n_qubits, w.ham.n_words
    eng = pe.Engine(0)
    if args.partition or args.partition_count:
        eng.set_tuning(partition=args.partition, partition_count=args.partition_count)
    eng.set_hamiltonian(N, w.ham.coeff, w.ham.xy, w.ham.yz)
    info = eng.info()
    G, NT = info["n_groups"], info["n_terms"]
    keys = torch.from_numpy(w.keys.view(np.int64)).cuda()
    L = torch.from_numpy(w.logpsi).cuda()
    Wt = None if w.weights is None else torch.from_numpy(w.weights).cuda()
    out = torch.empty(M, dtype=torch.complex128, device="cuda")
    stats = torch.empty(4, dtype=torch.float64, device="cuda")
    print(f"# workload {w.name}: N={N} M={M} terms={NT} groups={G} (set up in {time.perf_counter() - t0:.1f} s)",
          file=sys.stderr, flush=True)

    def make_step(variant, prec):
        def step():
            eng.set_samples(keys, check=False)
            eng.local_energy(L, Wt, variant, prec, out=out, stats=stats, check=False)
        return step

    order = [args.variant] + [v for v in ("terms", "batch", "trie") if v != args.variant and not args.only]
    res = {}
    for var in order:
        steps = args.steps if var == args.variant else min(args.steps, args.other_steps)
        warm = args.warmup if var == args.variant else min(args.warmup, 2)
        for prec in ("fp64", "fp32c"):
            ms, prof = time_steps(eng, make_step(var, prec), steps, warm)
            res.setdefault(var, {})[prec] = {
                "ms_per_step": ms, "steps": steps,
                "stage_ms": {k: v[0] / v[1] for k, v in prof.items() if v[1]},
                "eloc": out.cpu().numpy().copy(), "stats": stats.cpu().numpy().copy()}
            print(f"# {var} {prec}: {ms:.3f} ms/step  stages(ms/launch): " +
                  ", ".join(f"{k}={v[0] / v[1]:.3f}" for k, v in prof.items() if v[1]),
                  file=sys.stderr, flush=True)

    # work counts (outside the timed regions)
    sizes = group_sizes_by_id(w.ham)
    n_pairs = eng.count_pairs(args.variant)
    term_evals = term_evaluations(eng, args.variant, sizes)
    counts = {}
    for var in order:
        counts[var] = {"coupled_pairs": eng.count_pairs(var),
                       "candidates": M * G if var == "terms" else (M * M if var == "batch" else eng.trie_visits())}
        assert counts[var]["coupled_pairs"] == n_pairs, (var, counts[var], n_pairs)
    print(f"# {n_pairs} coupled pairs, {term_evals} term evaluations", file=sys.stderr, flush=True)

    head = res[args.variant]["fp32c"]
    fp64 = res[args.variant]["fp64"]
    pairs_s = n_pairs / (head["ms_per_step"] * 1e-3)

    traffic = measured_traffic(f"k_pairs_{w.name}_{args.variant}_fp32c_traffic.md")
    rooflines = {}
    for var in order:
        if counts[var]["candidates"] is None:
            continue
        for prec in ("fp64", "fp32c"):
            k_ms = res[var][prec]["stage_ms"]["pairs"]
            rooflines[f"{var}_{prec}"] = roofline(var, prec, W, M, NT, G, counts[var]["candidates"], term_evals,
                                                  n_pairs, k_ms * 1e-3,
                                                  traffic if (var, prec) == (args.variant, "fp32c") else None)
    roof = rooflines[f"{args.variant}_fp32c"]

    rec = {
        "metric": "coupled pairs/sec + E_loc^var samples/sec vs plain FP64 at |dE|<=1e-6 Ha",
        "value": pairs_s, "unit": "coupled pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32c", "data": "synthetic",
        "config": {"workload": f"{w.name}: {N} qubits, {w.n_electrons} electrons, {M} unique determinants, "
                               f"{NT} Pauli terms in {G} XY groups",
                   "variant": args.variant, "global_batch": M},
        "samples_per_s": M / (head["ms_per_step"] * 1e-3),
        "coupled_pairs": n_pairs, "candidates": counts[args.variant]["candidates"], "term_evaluations": term_evals,
        "fp64": {"pairs_per_s": n_pairs / (fp64["ms_per_step"] * 1e-3),
                 "samples_per_s": M / (fp64["ms_per_step"] * 1e-3), "ms_per_step": fp64["ms_per_step"]},
        "fp32c_over_fp64": fp64["ms_per_step"] / head["ms_per_step"],
        "roofline": roof,
        "variants": {var: {prec: {"ms_per_step": res[var][prec]["ms_per_step"], "steps": res[var][prec]["steps"],
                                  "pairs_per_s": n_pairs / (res[var][prec]["ms_per_step"] * 1e-3),
                                  "stage_ms": res[var][prec]["stage_ms"],
                                  "roofline_frac": rooflines.get(f"{var}_{prec}", {}).get("frac")}
                           for prec in ("fp64", "fp32c")} | {"candidates": counts[var]["candidates"]}
                     for var in order},
    }

    # accuracy against the oracle's stored results for this workload
    gold_path = GOLDEN / f"{w.name}_oracle.npz"
    if gold_path.exists():
        gold = dict(np.load(gold_path, allow_pickle=False))
        rows = gold["rows"]
        E_ref = gold["stats"][0] + 1j * gold["stats"][1]
        rec["accuracy"] = {"reference": f"oracle results stored in tests/golden/{gold_path.name} "
                                        f"({rows.size} sampled rows; E and Var over all rows)"}
        for var in order:
            for prec in ("fp64", "fp32c"):
                r = res[var][prec]
                rec["accuracy"][f"{var}_{prec}"] = {
                    "max_abs_dE_loc": float(np.abs(r["eloc"][rows] - gold["eloc"]).max()),
                    "abs_dE": float(abs(r["stats"][0] + 1j * r["stats"][1] - E_ref)),
                    "abs_dVar": float(abs(r["stats"][2] - gold["stats"][2]))}
        rec["energy"] = {"E": float(gold["stats"][0]), "Var": float(gold["stats"][2])}

    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w, res[args.variant])
    if not args.no_medium and w.name != "medium":
        eng.close()
        eng = None
        rec["medium"] = bench_medium(args)
    if not args.no_batched:
        rec["batched"] = bench_batched(args)
    if not args.no_adjoint:
        rec["adjoint"] = bench_adjoint(args)
    if not args.no_next:
        rec["full_local_energy"] = bench_full(args)
        rec["sr"] = bench_sr(args)
        rec["sampler"] = bench_sampler(args)
    if args.calibrate_mib:
        n = args.calibrate_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        rec["calibration_copy_bytes"] = 2 * n * 8
    print(json.dumps(rec))
    if eng is not None:
        eng.close()


def cpu_baseline(w, res_head):
    """The oracle (plain C, FP64, OpenMP over rows) on a bounded sample of
    rows of the same workload: all host threads, and one thread."""
    import numpy as np

    import oracle
    M = w.n_unique
    threads = oracle.max_threads()
    # about 10 s of oracle work each at the 52-qubit workload
    per_thread_rows = max(16, min(M // max(threads, 1), int(4096 * 16 / max(threads, 1)) // 16))
    rows_all = (0, min(M, per_thread_rows * threads))
    rows_one = (0, min(M, per_thread_rows))
    t0 = time.perf_counter()
    ref, npairs = oracle.local_energy(w.ham, w.keys, w.logpsi, rows=rows_all, with_pairs=True)
    t_all = time.perf_counter() - t0
    oracle.set_threads(1)
    t0 = time.perf_counter()
    _, npairs1 = oracle.local_energy(w.ham, w.keys, w.logpsi, rows=rows_one, with_pairs=True)
    t_one = time.perf_counter() - t0
    oracle.set_threads(threads)
    a, b = rows_all
    acc = {p: float(np.abs(res_head[p]["eloc"][a:b] - ref).max()) for p in ("fp64", "fp32c")}
    # the oracle on the other workloads (all host threads, bounded row samples)
    from synth import configs
    others = {}
    for name, rows in (("small", None), ("medium", 4096), ("wide", 128)):
        wo = getattr(configs, name)()
        r = (0, wo.n_unique if rows is None else min(wo.n_unique, rows))
        t0 = time.perf_counter()
        _, np_o = oracle.local_energy(wo.ham, wo.keys, wo.logpsi, rows=r, with_pairs=True)
        t_o = time.perf_counter() - t0
        others[name] = {"pairs_per_s": float(np_o.sum()) / t_o, "samples_per_s": (r[1] - r[0]) / t_o,
                        "sample": f"rows [{r[0]}, {r[1]}) of {wo.n_unique} ({wo.n_qubits} qubits), {t_o:.2f} s wall"}
    return {"value": float(npairs.sum()) / t_all, "unit": "coupled pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"rows [{a}, {b}) of the workload ({b - a} of {M} samples, {int(npairs.sum())} coupled "
                      f"pairs), one forward pass, {t_all:.2f} s wall on {threads} threads",
            "samples_per_s": (b - a) / t_all,
            "single_thread": {"value": float(npairs1.sum()) / t_one, "unit": "coupled pairs/s",
                              "sample": f"rows [{rows_one[0]}, {rows_one[1]}), {t_one:.2f} s wall",
                              "samples_per_s": (rows_one[1] - rows_one[0]) / t_one},
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "gpu_vs_oracle_max_abs_dE_loc": acc, "other_workloads": others}


def bench_medium(args):
    """28 qubits, 65 536 samples: LoopOverTerms, both precisions."""
    import numpy as np
    import torch

    import paper_2408_07625_amd as pe
    from synth import configs

    w = configs.medium()
    M, N, W = w.n_unique, w.n_qubits, w.ham.n_words
    eng = pe.Engine(0)
    eng.set_hamiltonian(N, w.ham.coeff, w.ham.xy, w.ham.yz)
    info = eng.info()
    keys = torch.from_numpy(w.keys.view(np.int64)).cuda()
    L = torch.from_numpy(w.logpsi).cuda()
    out = torch.empty(M, dtype=torch.complex128, device="cuda")
    stats = torch.empty(4, dtype=torch.float64, device="cuda")
    r = {"workload": f"medium: {N} qubits, {w.n_electrons} electrons, {M} unique determinants, "
                     f"{info['n_terms']} Pauli terms in {info['n_groups']} XY groups", "variant": "terms"}
    for prec in ("fp64", "fp32c"):
        def step():
            eng.set_samples(keys, check=False)
            eng.local_energy(L, None, "terms", prec, out=out, stats=stats, check=False)
        ms, prof = time_steps(eng, step, args.steps, args.warmup)
        r[prec] = {"ms_per_step": ms, "stage_ms": {k: v[0] / v[1] for k, v in prof.items() if v[1]}}
    n_pairs = eng.count_pairs("terms")
    te = term_evaluations(eng, "terms", group_sizes_by_id(w.ham))
    r["coupled_pairs"] = n_pairs
    for prec in ("fp64", "fp32c"):
        r[prec]["pairs_per_s"] = n_pairs / (r[prec]["ms_per_step"] * 1e-3)
        rf = roofline("terms", prec, W, M, info["n_terms"], info["n_groups"], M * info["n_groups"], te, n_pairs,
                      r[prec]["stage_ms"]["pairs"] * 1e-3, None)
        r[prec]["roofline_frac"] = rf["frac"]
    print(f"# medium: fp64 {r['fp64']['ms_per_step']:.3f} ms, fp32c {r['fp32c']['ms_per_step']:.3f} ms",
          file=sys.stderr, flush=True)
    eng.close()
    return r


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
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


def bench_full(args):
    """Conventional local energy (Eq. local_energy over every coupled x') on
    the 28-qubit workload: the list of coupled states outside U, then E_loc
    over U and them; their log-amplitudes are synthetic (the recipe's rank
    law), as an ansatz would supply them."""
    import numpy as np
    import torch

    import paper_2408_07625_amd as pe
    from synth import configs, samples

    w = configs.medium()
    eng = pe.Engine(0)
    eng.set_hamiltonian(w.n_qubits, w.ham.coeff, w.ham.xy, w.ham.yz)
    keys = torch.from_numpy(w.keys.view(np.int64)).cuda()
    eng.set_samples(keys)
    L = torch.from_numpy(w.logpsi).cuda()
    steps = max(1, min(args.steps, args.other_steps))
    # the library keeps the last list for unchanged samples: time the list
    # from fresh samples (set_samples + find_misses) less set_samples alone
    t_set = _timed(lambda: eng.set_samples(keys), steps, 1)
    t_set_find = _timed(lambda: (eng.set_samples(keys), eng.find_misses()), steps, 1)
    t_find = t_set_find - t_set
    V = eng.find_misses()
    Vn = V.cpu().numpy().view(np.uint64)
    rank = samples.excitation_rank(Vn, w.n_qubits, w.n_electrons)
    rng = np.random.default_rng(11)
    Lv = torch.from_numpy(samples.log_amplitudes(rank, rng)).cuda()
    res = {"workload": f"medium: {w.n_qubits} qubits, {w.n_unique} samples; {V.shape[0]} coupled states outside U",
           "extra_states": int(V.shape[0]), "find_ms": t_find, "set_samples_plus_find_ms": t_set_find}
    for prec in ("fp64", "fp32c"):
        res[prec] = {"ms": _timed(lambda: eng.local_energy_full(L, V, Lv, None, prec), steps, 1)}
    e_full, st_full = eng.local_energy_full(L, V, Lv, None, "fp64")
    e_var, st_var = eng.local_energy(L, None, "terms", "fp64")
    res["E_full"] = float(st_full[0].item())
    res["E_var"] = float(st_var[0].item())
    print(f"# full local energy: {V.shape[0]} extra states, find {t_find:.2f} ms, "
          f"E_loc {res['fp64']['ms']:.2f} / {res['fp32c']['ms']:.2f} ms", file=sys.stderr, flush=True)
    eng.close()
    return res


def bench_sr(args):
    """SR step at the paper's working point: N_SR = 100 samples, a parameter
    vector of the size of its ansatz at 52 qubits (9 qudits of 6 qubits, two
    perceptrons of width 64 each: 210 816 parameters), synthetic Jacobian."""
    import numpy as np
    import torch

    import paper_2408_07625_amd as pe
    n_sr, n_p = 100, 210_816
    rng = np.random.default_rng(12)
    O_re = torch.from_numpy(rng.normal(size=(n_sr, n_p))).cuda()
    O_im = torch.from_numpy(rng.normal(size=(n_sr, n_p))).cuda()
    L = torch.from_numpy(rng.normal(size=n_sr) + 1j * rng.uniform(0, 6, n_sr)).cuda()
    F = torch.from_numpy(rng.normal(size=n_p)).cuda()
    M = 1 << 20
    Lu = torch.from_numpy(rng.normal(size=M) + 1j * rng.uniform(0, 6, M)).cuda()
    eng = pe.Engine(0)
    out = torch.empty(n_p, dtype=torch.float64, device="cuda")
    steps = max(2, min(args.steps, 10))
    ms = _timed(lambda: eng.sr_solve(O_re, O_im, L, F, 1e-3, out=out, check=False), steps, 2)
    eng.check()
    sel = _timed(lambda: eng.sr_select(Lu, n_sr), steps, 2)
    R = 2 * n_sr + 1
    flops = R * R * n_p          # Gram of the centred rows (upper triangle: half of 2 R^2 N_p)
    bytes_ = 2 * (2 * n_sr * n_p * 8) + 3 * n_p * 8   # the Jacobian read twice, F, mean, d
    res = {"workload": f"N_SR = {n_sr}, {n_p} parameters, lambda = 1e-3; selection from 2^20 samples",
           "solve_ms": ms, "select_ms": sel,
           "gram_fp64_tflops_effective": flops / (ms * 1e-3) / 1e12,
           "hbm_gb_s_effective": bytes_ / (ms * 1e-3) / 1e9}
    print(f"# sr: solve {ms:.3f} ms, select {sel:.3f} ms", file=sys.stderr, flush=True)
    eng.close()
    return res


def bench_sampler(args):
    """ARGumbelTopK: 2^16 unique samples of 52 qubits (9 qudits of 6),
    (10, 10) electrons, perceptrons of width 64 with random weights."""
    import numpy as np
    import torch

    import paper_2408_07625_amd as pe
    N, D, K = 52, 6, 1 << 16
    Q = (N + D - 1) // D
    rng = np.random.default_rng(13)
    wts = {"W1": rng.normal(scale=1.5 / np.sqrt(N), size=(Q, 64, N)), "b1": rng.normal(scale=0.1, size=(Q, 64)),
           "W2": rng.normal(scale=1.5 / 8, size=(Q, 64, 64)), "b2": rng.normal(scale=0.1, size=(Q, 64)),
           "W3": rng.normal(scale=1.5 / 8, size=(Q, 64, 64)), "b3": rng.normal(scale=0.5, size=(Q, 64))}
    wts = {k: torch.from_numpy(v).cuda() for k, v in wts.items()}
    eng = pe.Engine(0)
    steps = max(2, min(args.steps, args.other_steps))
    ms = _timed(lambda: eng.sample(N, D, wts, K, seed=5, n_up=10, n_down=10), steps, 1)
    keys, logp, _ = eng.sample(N, D, wts, K, seed=5, n_up=10, n_down=10)
    res = {"workload": f"{N} qubits, qudits of {D}, (10, 10) electrons, K = {K}", "ms": ms,
           "samples": int(keys.shape[0]), "samples_per_s": keys.shape[0] / (ms * 1e-3)}
    print(f"# sampler: {ms:.2f} ms for {keys.shape[0]} samples", file=sys.stderr, flush=True)
    eng.close()
    return res


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
    steps = max(2, min(args.steps, args.other_steps))

    def timed(fn):
        for _ in range(max(1, min(args.warmup, 2))):
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
        b.profile(True)
        b.profile_read()
        ms_eager = timed(lambda: b.run(prec, check=False), args.steps)
        b.check()
        prof = b.profile_read()
        b.profile(False)
        b.set_graph(True)
        out[prec] = {"ms_per_step": ms, "pairs_per_s": pairs / (ms * 1e-3), "samples_per_s": S / (ms * 1e-3),
                     "eager_ms_per_step": ms_eager,
                     "eager_stage_ms": {k: v[0] / v[1] for k, v in prof.items() if v[1]}}
        out["coupled_pairs"] = pairs
        print(f"# batched {prec}: graph {ms:.3f} ms, eager {ms_eager:.3f} ms, {pairs} pairs, stages "
              + ", ".join(f"{k}={v[0] / max(v[1], 1):.3f}" for k, v in prof.items()), file=sys.stderr, flush=True)
    # the same problems one by one: one context each (Hamiltonian ingested
    # once), each step sets the samples and runs the forward pass
    engines = []
    cand, te, pairs_k = 0, 0, 0
    for k, w in enumerate(ws):
        e = pe.Engine(0)
        e.set_hamiltonian(w.n_qubits, w.ham.coeff, w.ham.xy, w.ham.yz)
        info = b.problem_info(k)
        engines.append((e, info["variant"], probs[k]["keys"], probs[k]["logpsi"],
                        torch.empty(w.n_unique, dtype=torch.complex128, device="cuda"),
                        torch.empty(4, dtype=torch.float64, device="cuda")))
        # work counts of the batched pair kernel, per problem
        e.set_samples(probs[k]["keys"])
        Wk = w.ham.n_words
        cand += w.n_unique * (info["n_groups"] * ops_per_candidate("terms", Wk) if info["variant"] == "terms"
                              else w.n_unique * ops_per_candidate("batch", Wk))
        te += term_evaluations(e, info["variant"], group_sizes_by_id(w.ham))
        pairs_k += e.count_pairs(info["variant"])
    assert pairs_k == out["coupled_pairs"], (pairs_k, out["coupled_pairs"])

    def sequential(prec):
        for e, var, keys, L, o, s in engines:
            e.set_samples(keys, check=False)
            e.local_energy(L, None, var, prec, out=o, stats=s, check=False)

    for prec in ("fp32c", "fp64"):
        ms = timed(lambda: sequential(prec), max(1, args.steps // 4))
        out[prec]["sequential_ms_per_step"] = ms
        out[prec]["speedup_vs_sequential"] = ms / out[prec]["ms_per_step"]
        print(f"# sequential {prec}: {ms:.3f} ms", file=sys.stderr, flush=True)
        ops = cand + te * OPS_PER_TERM + pairs_k * OPS_PER_PAIR[prec]
        k_s = out[prec]["eager_stage_ms"]["pairs"] * 1e-3
        out[prec]["roofline"] = {"bound": "alu", "achieved": ops / k_s / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                                 "unit": "Tlane-op/s", "frac": ops / k_s / PEAK_LANE_OPS,
                                 "kernel": "k_pairs_batched (both key formats), eager launch",
                                 "kernel_ms": k_s * 1e3, "ops_per_launch": ops}
    out["term_evaluations"] = te
    out["fp32c_over_fp64"] = out["fp64"]["ms_per_step"] / out["fp32c"]["ms_per_step"]
    for e, *_ in engines:
        e.close()
    b.close()
    return out


if __name__ == "__main__":
    main()
