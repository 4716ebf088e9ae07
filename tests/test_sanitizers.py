"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the oracle's C source and the prefix-tree construction / walk shared
with the GPU kernels (csrc/trie.h) are compiled with both sanitizers and run
on small inputs in a child process that preloads the sanitizer runtime; any
report fails the test."""
import os
import subprocess
import sys
from pathlib import Path

import pytest

HERE = Path(__file__).resolve().parent
ROOT = HERE.parent
BUILD = HERE / "host" / "_build"

SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined", "-g", "-O1"]

ORACLE_SCRIPT = r"""
import numpy as np
import oracle
from oracle import sr
from synth import jw
rng = np.random.default_rng(0)
for N, T, W2 in ((9, 120, False), (70, 60, True)):
    ham = jw.random_pauli(N, T, rng, max_flip=3)
    if W2:
        keys = rng.integers(0, 2 ** 62, size=(40, 2), dtype=np.int64).astype(np.uint64)
        keys[:, 1] &= np.uint64((1 << (N - 64)) - 1)
        keys = np.unique(keys, axis=0)
    else:
        keys = rng.choice(2 ** N, 60, replace=False).astype(np.uint64)[:, None]
    M = keys.shape[0]
    L = rng.normal(size=M) + 1j * rng.normal(size=M)
    e = oracle.local_energy(ham, keys, L)
    oracle.find_pairs(ham, keys, rows=(0, M), with_elements=True)
    oracle.phase_exponents(ham, keys[:10], keys[10:20])
    oracle.matrix_elements(ham, keys[:10], keys[5:15])
    E, var, _ = oracle.energy(e, L)
    oracle.adjoint(ham, keys, L, e, 1.0 + 0.5j, energy_value=E)
    V = oracle.find_misses(ham, keys)
    oracle.local_energy_full(ham, keys, L, V, np.zeros(V.shape[0], complex))
print("oracle ok")
"""


def _run(env_extra, script, *argv):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=23"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1:exitcode=24"
    env["PYTHONPATH"] = str(ROOT) + os.pathsep + env.get("PYTHONPATH", "")
    return subprocess.run([sys.executable, "-c", script, *argv], env=env, capture_output=True, text=True,
                          timeout=600)


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    if not path or not Path(path).exists():
        pytest.skip(f"{name} not available")
    return path


def test_oracle_under_asan_ubsan():
    BUILD.mkdir(parents=True, exist_ok=True)
    lib = BUILD / "liboracle_san.so"
    subprocess.run(["gcc", *SAN, "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", str(lib),
                    str(ROOT / "oracle" / "eloc_oracle.c"), "-lm"], check=True)
    r = _run({"ORACLE_LIB": str(lib), "LD_PRELOAD": _runtime("libasan.so") + " " + _runtime("libubsan.so"),
              "OMP_NUM_THREADS": "2"}, ORACLE_SCRIPT)
    assert r.returncode == 0 and "oracle ok" in r.stdout, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])


TRIE_SCRIPT = r"""
import ctypes, sys
import numpy as np
L = ctypes.CDLL(sys.argv[1])
L.trie_pairs_host.restype = ctypes.c_int64
L.trie_pairs_host.argtypes = [ctypes.c_int] + [ctypes.c_void_p, ctypes.c_int64] * 3 + [ctypes.c_int64] + [ctypes.c_void_p] * 4
rng = np.random.default_rng(1)
p = lambda a: ctypes.c_void_p(a.ctypes.data)
for W, nu, nv, nx in ((1, 1, 1, 3), (1, 2, 1, 5), (1, 300, 40, 50), (2, 200, 30, 40), (1, 1, 64, 10)):
    hi = 2 ** 40 if W == 1 else 2 ** 62
    U = np.unique(rng.integers(0, hi, size=(nu, W), dtype=np.int64).astype(np.uint64), axis=0)
    V = np.unique(rng.integers(0, 2 ** 12, size=(nv, W), dtype=np.int64).astype(np.uint64), axis=0)
    U = U[np.lexsort(tuple(U[:, w] for w in range(W)))]
    V = V[np.lexsort(tuple(V[:, w] for w in range(W)))]
    X = U[rng.integers(0, U.shape[0], size=nx)] ^ V[rng.integers(0, V.shape[0], size=nx)]
    X = np.ascontiguousarray(X)
    cap = U.shape[0] * X.shape[0] + 1
    r = np.zeros(cap, np.int64); u = np.zeros(cap, np.int64); v = np.zeros(cap, np.int64)
    nodes = np.zeros(4 * max(U.shape[0], 1), np.int32)
    n = L.trie_pairs_host(W, p(U), U.shape[0], p(V), V.shape[0], p(X), X.shape[0], cap, p(r), p(u), p(v), p(nodes))
    assert n >= nx
print("trie ok")
"""


def test_trie_host_code_under_asan_ubsan():
    BUILD.mkdir(parents=True, exist_ok=True)
    lib = BUILD / "libtriecheck_san.so"
    src = HERE / "host" / "trie_check.cpp"
    hdr = ROOT / "paper_2408_07625_amd" / "csrc"
    # host-only build of the shared templates with g++ (no GPU code on this line)
    r = subprocess.run(["g++", *SAN, "-std=c++17", "-fPIC", "-shared", "-D__HIP_PLATFORM_AMD__",
                        "-I/opt/rocm/include", f"-I{hdr}", str(src), "-o", str(lib)], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("trie_check.cpp needs hipcc's host compiler: " + r.stderr[-300:])
    r = _run({"LD_PRELOAD": _runtime("libasan.so") + " " + _runtime("libubsan.so")}, TRIE_SCRIPT, str(lib))
    assert r.returncode == 0 and "trie ok" in r.stdout, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
