"""spin_split, the bit permutation behind the LoopOverTerms prefilter of
wide keys, compiled for the host from the same header the kernels include
and checked bit by bit: even qubits (spin up under the interleaved
Jordan-Wigner order) in order in the low half, odd ones in the high half."""
import ctypes
import subprocess
from pathlib import Path

import numpy as np
import pytest

HERE = Path(__file__).resolve().parent
ROOT = HERE.parent
SRC = HERE / "host" / "split_check.cpp"
HDR = ROOT / "paper_2408_07625_amd" / "csrc" / "internal.h"
OUT = HERE / "host" / "_build" / "libsplitcheck.so"


@pytest.fixture(scope="module")
def split():
    OUT.parent.mkdir(exist_ok=True)
    if not OUT.exists() or OUT.stat().st_mtime < max(SRC.stat().st_mtime, HDR.stat().st_mtime):
        subprocess.run(["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-fPIC", "-shared",
                        f"-I{HDR.parent}", f"-I{ROOT / 'include'}", str(SRC), "-o", str(OUT)],
                       check=True, capture_output=True)
    L = ctypes.CDLL(str(OUT))
    L.spin_split_host.restype = None
    L.spin_split_host.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]

    def f(x):
        x = np.ascontiguousarray(x, dtype=np.uint64)
        out = np.empty_like(x)
        L.spin_split_host(x.ctypes.data, x.size, out.ctypes.data)
        return out
    return f


def bits(x):
    return ((x[:, None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)).astype(np.uint8)


def test_layout(split):
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.integers(0, 2**63, size=4000, dtype=np.uint64) * np.uint64(2)
                        + rng.integers(0, 2, size=4000, dtype=np.uint64),
                        np.array([0, 2**64 - 1, 0x5555555555555555, 0xAAAAAAAAAAAAAAAA, 1, 2**63],
                                 dtype=np.uint64)])
    b, s = bits(x), bits(split(x))
    np.testing.assert_array_equal(s[:, :32], b[:, 0::2])
    np.testing.assert_array_equal(s[:, 32:], b[:, 1::2])


def test_prefilter_counts(split):
    """The counts the filter takes from the permuted XOR equal the sector
    popcounts of the plain XOR (the permutation commutes with XOR)."""
    rng = np.random.default_rng(6)
    a = rng.integers(0, 2**63, size=5000, dtype=np.uint64)
    g = rng.integers(0, 2**63, size=5000, dtype=np.uint64)
    s = split(a) ^ split(g)
    np.testing.assert_array_equal(split(a ^ g), s)
    even = np.bitwise_count((a ^ g) & np.uint64(0x5555555555555555))
    odd = np.bitwise_count((a ^ g) & np.uint64(0xAAAAAAAAAAAAAAAA))
    np.testing.assert_array_equal(np.bitwise_count(s & np.uint64(0xFFFFFFFF)), even)
    np.testing.assert_array_equal(np.bitwise_count(s >> np.uint64(32)), odd)
