"""The prefix-tree construction and dual walk of the LoopOverTrie kernels,
compiled for the host and checked against brute force on the CPU.

The same templates (csrc/trie.h) are instantiated by the GPU kernels; this
test exercises their indexing (node ranges, leaf encoding, stack bound) on
small and edge-case inputs before any GPU run.
"""
import ctypes
import subprocess
from pathlib import Path

import numpy as np
import pytest

HERE = Path(__file__).resolve().parent
ROOT = HERE.parent
SRC = HERE / "host" / "trie_check.cpp"
HDR = ROOT / "paper_2408_07625_amd" / "csrc" / "trie.h"
OUT = HERE / "host" / "_build" / "libtriecheck.so"


@pytest.fixture(scope="module")
def lib():
    OUT.parent.mkdir(exist_ok=True)
    if not OUT.exists() or OUT.stat().st_mtime < max(SRC.stat().st_mtime, HDR.stat().st_mtime):
        subprocess.run(["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-fPIC", "-shared",
                        f"-I{HDR.parent}", str(SRC), "-o", str(OUT)], check=True, capture_output=True)
    L = ctypes.CDLL(str(OUT))
    L.trie_pairs_host.restype = ctypes.c_int64
    L.trie_pairs_host.argtypes = [ctypes.c_int] + [ctypes.c_void_p, ctypes.c_int64] * 3 + \
        [ctypes.c_int64] + [ctypes.c_void_p] * 4
    return L


def sorted_keys(keys):
    W = keys.shape[1]
    order = np.lexsort(tuple(keys[:, w] for w in range(W)))   # last key (top word) primary
    return keys[order]


def walk(lib, U, V, X):
    W = U.shape[1]
    cap = U.shape[0] * X.shape[0] + 1
    r = np.zeros(cap, np.int64)
    u = np.zeros(cap, np.int64)
    v = np.zeros(cap, np.int64)
    nodes = np.zeros(4 * max(U.shape[0], 1), np.int32)
    p = lambda a: ctypes.c_void_p(a.ctypes.data)
    n = lib.trie_pairs_host(W, p(U), U.shape[0], p(V), V.shape[0], p(X), X.shape[0], cap, p(r), p(u), p(v),
                            p(nodes))
    return set(zip(r[:n].tolist(), u[:n].tolist(), v[:n].tolist())), n, nodes.reshape(-1, 4)


def brute(U, V, X):
    vset = {tuple(k): i for i, k in enumerate(V.tolist())}
    out = set()
    for r, x in enumerate(X):
        for ui, k in enumerate(U):
            m = tuple((x ^ k).tolist())
            if m in vset:
                out.add((r, ui, vset[m]))
    return out


def rand_keys(rng, n, nbits, W, maxpop=None):
    keys = set()
    while len(keys) < n:
        if maxpop is None:
            bits = rng.random(nbits) < 0.5
        else:
            bits = np.zeros(nbits, bool)
            bits[rng.choice(nbits, size=rng.integers(0, maxpop + 1), replace=False)] = True
        keys.add(tuple(sum(1 << (int(q) - 64 * w) for q in np.flatnonzero(bits) if 64 * w <= q < 64 * w + 64)
                       for w in range(W)))
    return np.array(sorted(keys), dtype=np.uint64).reshape(n, W)


@pytest.mark.parametrize("W,nbits,nU,nV", [(1, 6, 20, 10), (1, 12, 200, 80), (1, 64, 300, 100),
                                           (2, 100, 150, 60), (2, 128, 64, 64), (1, 8, 1, 5), (1, 8, 5, 1),
                                           (1, 8, 1, 1), (1, 8, 2, 2)])
def test_walk_matches_brute_force(lib, W, nbits, nU, nV):
    rng = np.random.default_rng(nbits * 1000 + nU)
    U = sorted_keys(rand_keys(rng, nU, nbits, W))
    V = sorted_keys(rand_keys(rng, nV, nbits, W, maxpop=4))
    X = np.concatenate([U, rand_keys(rng, 10, nbits, W)])
    got, n, _ = walk(lib, U, V, X)
    assert n == len(got)            # no pair reported twice
    assert got == brute(U, V, X)


def test_dense_coupling(lib):
    """Every XOR is in the XY set: the walk must enumerate all of U x U."""
    U = sorted_keys(np.arange(64, dtype=np.uint64)[:, None])
    got, n, _ = walk(lib, U, U, U)
    assert n == 64 * 64 and got == brute(U, U, U)


def test_node_ranges(lib):
    rng = np.random.default_rng(2)
    U = sorted_keys(rand_keys(rng, 50, 20, 1))
    _, _, nodes = walk(lib, U, U[:1], U[:1])
    n = U.shape[0]
    nodes = nodes[: n - 1]
    # every leaf is reached exactly once from the root, and every internal node
    # except the root has exactly one parent
    seen_leaf = np.zeros(n, int)
    seen_node = np.zeros(n - 1, int)
    for nd in nodes:
        for ch in nd[:2]:
            if ch < 0:
                seen_leaf[~ch] += 1
            else:
                seen_node[ch] += 1
    assert (seen_leaf == 1).all() and seen_node[0] == 0 and (seen_node[1:] == 1).all()
    # the branch bit separates the two children
    for i, nd in enumerate(nodes):
        b = nd[3]
        assert ((int(U[nd[2], 0]) >> b) & 1) in (0, 1)
