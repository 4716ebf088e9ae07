"""Write tests/golden/large_oracle.npz: oracle results for the 52-qubit
workload (20 electrons, 2^20 unique determinants), computed by the CPU
oracle only.

    python tests/golden/make_large_golden.py [--threads T]

Contents (numeric arrays only; np.load with allow_pickle=False reads them):

  rows         int64 [R]   sampled rows: the first and last 1024, and 14
                           blocks of 768 at seeded random offsets (R = 12800)
  eloc         complex128 [R]  E_loc^var of those rows
  count        int64 [R]   coupled samples of each row (diagonal included)
  digest       uint64 [R]  order-independent digest of the row's (j, g)
                           pairs (tests/digest.py)
  stats        float64 [4] Re E, Im E, Var, sum of raw weights over all rows
                           (|psi|^2 weights)
  total_pairs  int64 []    coupled ordered pairs over all rows
  fingerprint  uint8 [32]  SHA-256 of the generated inputs, so that a change
                           of the generator fails the tests loudly

The full pass over all rows takes about 40 minutes on eight cores.
"""
from __future__ import annotations

import argparse
import hashlib
import sys
import time
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
ROOT = HERE.parent.parent
sys.path.insert(0, str(ROOT))
sys.path.insert(0, str(HERE.parent))

OUT = HERE / "large_oracle.npz"


def fingerprint(w) -> np.ndarray:
    h = hashlib.sha256()
    for a in (w.ham.coeff, w.ham.xy, w.ham.yz, w.keys, w.logpsi):
        h.update(np.ascontiguousarray(a).tobytes())
    return np.frombuffer(h.digest(), dtype=np.uint8).copy()


def sample_blocks(M: int, seed: int = 20240807):
    """Row blocks [a, b): the first and last 1024 rows, then 14 disjoint
    blocks of 768 rows at seeded random offsets between them."""
    blocks = [(0, 1024), (M - 1024, M)]
    rng = np.random.default_rng(seed)
    span = (M - 2048) // 14
    for k in range(14):
        a = 1024 + k * span + int(rng.integers(0, span - 768))
        blocks.append((a, a + 768))
    return sorted(blocks)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args()

    import oracle
    from digest import row_digests
    from synth import configs

    if args.threads:
        oracle.set_threads(args.threads)
    t0 = time.time()
    w = configs.large()
    M = w.n_unique
    print(f"inputs: {w.n_qubits} qubits, {M} samples, {w.ham.n_terms} terms ({time.time() - t0:.1f} s)",
          flush=True)
    blocks = sample_blocks(M)
    rows, counts, digests = [], [], []
    for a, b in blocks:
        t = time.time()
        pi, pj, pg = oracle.find_pairs(w.ham, w.keys, rows=(a, b))
        r = np.arange(a, b, dtype=np.int64)
        c, d = row_digests(pi, pj, pg, r)
        rows.append(r)
        counts.append(c)
        digests.append(d)
        print(f"pairs of rows [{a}, {b}): {pi.size} ({time.time() - t:.1f} s)", flush=True)
    rows = np.concatenate(rows)
    counts = np.concatenate(counts)
    digests = np.concatenate(digests)

    t = time.time()
    eloc, npairs = oracle.local_energy(w.ham, w.keys, w.logpsi, with_pairs=True)
    print(f"full pass: {time.time() - t:.1f} s", flush=True)
    assert np.array_equal(npairs[rows], counts), "pair counts of the two oracle passes differ"
    E, var, tot = oracle.energy(eloc, w.logpsi, w.weights)
    np.savez_compressed(OUT, rows=rows, eloc=eloc[rows], count=counts, digest=digests,
                        stats=np.array([E.real, E.imag, var, tot]), total_pairs=np.int64(npairs.sum()),
                        fingerprint=fingerprint(w))
    print(f"wrote {OUT}: E = {E.real:.12f}, Var = {var:.6f}, pairs = {int(npairs.sum())}", flush=True)


if __name__ == "__main__":
    main()
