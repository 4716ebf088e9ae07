"""CPU FP64 oracle for the sample-aware local energy (test infrastructure).

TEST INFRASTRUCTURE ONLY: the correctness reference for the GPU library.
Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package; the library and its Python binding never do.

The computation lives in eloc_oracle.c (plain C, OpenMP over rows); this
module compiles it with gcc and marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "eloc_oracle.c"
_LIB = _HERE / "liboracle.so"
_lib = None


def build(force: bool = True) -> Path:
    """Compile liboracle.so next to the source."""
    if not force and _LIB.exists() and _LIB.stat().st_mtime >= _SRC.stat().st_mtime:
        return _LIB
    tmp = _LIB.with_suffix(".so.tmp")
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                    "-o", str(tmp), str(_SRC), "-lm"], check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        # ORACLE_LIB: a separately built copy (the sanitizer test's build)
        alt = os.environ.get("ORACLE_LIB")
        if alt:
            _lib = ctypes.CDLL(alt)
        else:
            build(force=False)
            _lib = ctypes.CDLL(str(_LIB))
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        _lib.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib.oracle_set_threads.restype = None
        _lib.oracle_max_threads.restype = ctypes.c_int
        _lib.oracle_groups.restype = i64
        _lib.oracle_groups.argtypes = [ctypes.c_int, i64, P, P]
        _lib.oracle_local_energy.restype = ctypes.c_int
        _lib.oracle_local_energy.argtypes = [ctypes.c_int, i64, P, P, P, i64, P, P, i64, i64, P, P]
        _lib.oracle_find_pairs.restype = ctypes.c_int
        _lib.oracle_find_pairs.argtypes = [ctypes.c_int, i64, P, P, P, i64, P, i64, i64, i64,
                                           P, P, P, P, P]
        _lib.oracle_matrix_elements.restype = ctypes.c_int
        _lib.oracle_matrix_elements.argtypes = [ctypes.c_int, i64, P, P, P, i64, P, P, P]
        _lib.oracle_phase_exponents.restype = i64
        _lib.oracle_phase_exponents.argtypes = [ctypes.c_int, i64, P, P, i64, P, P, P, P, i64]
        _lib.oracle_energy.restype = ctypes.c_int
        _lib.oracle_energy.argtypes = [i64, P, P, P, P]
        _lib.oracle_adjoint.restype = ctypes.c_int
        _lib.oracle_adjoint.argtypes = [ctypes.c_int, i64, P, P, P, i64, P, P, P, P, P,
                                        ctypes.c_double, ctypes.c_double, i64, i64, P]
        _lib.oracle_find_misses.restype = i64
        _lib.oracle_find_misses.argtypes = [ctypes.c_int, i64, P, P, P, i64, P, ctypes.c_double,
                                            ctypes.POINTER(ctypes.POINTER(ctypes.c_uint64))]
        _lib.oracle_free.argtypes = [P]
        _lib.oracle_free.restype = None
        _lib.oracle_local_energy_full.restype = ctypes.c_int
        _lib.oracle_local_energy_full.argtypes = [ctypes.c_int, i64, P, P, P, i64, P, P, i64, P, P,
                                                  ctypes.c_double, i64, i64, P]
    return _lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _ham_arrays(ham):
    c = np.ascontiguousarray(ham.coeff, dtype=np.float64)
    xy = np.ascontiguousarray(ham.xy, dtype=np.uint64)
    yz = np.ascontiguousarray(ham.yz, dtype=np.uint64)
    return c, xy, yz


class OracleError(RuntimeError):
    pass


def _check(rc):
    if rc == -2:
        raise OracleError("duplicate keys in U")
    if rc != 0:
        raise OracleError(f"oracle error {rc}")


def set_threads(n: int) -> None:
    """Number of OpenMP threads the oracle uses from now on."""
    _load().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def groups(ham) -> np.ndarray:
    """First-appearance group id of every term (unique XY set order)."""
    lib = _load()
    xy = np.ascontiguousarray(ham.xy, dtype=np.uint64)
    out = np.empty(ham.n_terms, dtype=np.int64)
    G = lib.oracle_groups(ham.n_qubits, ham.n_terms, _p(xy), _p(out))
    if G < 0:
        raise OracleError("bad Hamiltonian")
    return out


def local_energy(ham, keys, logpsi, rows=None, with_pairs=False):
    """E_loc^var (complex128) for rows [a, b) of U, caller order."""
    lib = _load()
    c, xy, yz = _ham_arrays(ham)
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    lp = np.ascontiguousarray(logpsi, dtype=np.complex128)
    a, b = (0, keys.shape[0]) if rows is None else rows
    out = np.empty(b - a, dtype=np.complex128)
    npairs = np.empty(b - a, dtype=np.int64)
    _check(lib.oracle_local_energy(ham.n_qubits, ham.n_terms, _p(c), _p(xy), _p(yz),
                                   keys.shape[0], _p(keys), _p(lp), a, b, _p(out), _p(npairs)))
    return (out, npairs) if with_pairs else out


def find_pairs(ham, keys, rows=None, with_elements=False):
    """Coupled pairs (i, j, g) sorted by (i, j) for rows [a, b), optionally H_ij."""
    lib = _load()
    c, xy, yz = _ham_arrays(ham)
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    a, b = (0, keys.shape[0]) if rows is None else rows
    n = ctypes.c_int64(0)
    cap = 0
    while True:
        pi = np.empty(max(cap, 1), dtype=np.int32)
        pj = np.empty(max(cap, 1), dtype=np.int32)
        pg = np.empty(max(cap, 1), dtype=np.int32)
        hij = np.empty(max(cap, 1), dtype=np.complex128) if with_elements else None
        _check(lib.oracle_find_pairs(ham.n_qubits, ham.n_terms, _p(c), _p(xy), _p(yz),
                                     keys.shape[0], _p(keys), a, b, cap, _p(pi), _p(pj), _p(pg),
                                     _p(hij), ctypes.byref(n)))
        if n.value <= cap:
            break
        cap = n.value
    k = n.value
    res = (pi[:k], pj[:k], pg[:k])
    return res + (hij[:k],) if with_elements else res


def matrix_elements(ham, x, xprime):
    lib = _load()
    c, xy, yz = _ham_arrays(ham)
    x = np.ascontiguousarray(x, dtype=np.uint64)
    xp = np.ascontiguousarray(xprime, dtype=np.uint64)
    out = np.empty(x.shape[0], dtype=np.complex128)
    _check(lib.oracle_matrix_elements(ham.n_qubits, ham.n_terms, _p(c), _p(xy), _p(yz),
                                      x.shape[0], _p(x), _p(xp), _p(out)))
    return out


def phase_exponents(ham, x, xprime):
    """(offsets int64 [n + 1], k uint8 [offsets[n]]): for pair p the
    exponent k of <x|P_l|x'> = i^k of every term l of the group of x ^ x',
    in ascending caller index (Eq. pauli_melem); no terms if x ^ x' is not
    an XY mask of H."""
    lib = _load()
    c, xy, yz = _ham_arrays(ham)
    x = np.ascontiguousarray(x, dtype=np.uint64)
    xp = np.ascontiguousarray(xprime, dtype=np.uint64)
    n = x.shape[0]
    off = np.empty(n + 1, dtype=np.int64)
    total = lib.oracle_phase_exponents(ham.n_qubits, ham.n_terms, _p(xy), _p(yz), n, _p(x), _p(xp), _p(off),
                                       None, 0)
    if total < 0:
        raise OracleError("bad Hamiltonian")
    k = np.empty(max(total, 1), dtype=np.uint8)
    lib.oracle_phase_exponents(ham.n_qubits, ham.n_terms, _p(xy), _p(yz), n, _p(x), _p(xp), _p(off), _p(k), total)
    return off, k[:total]


def energy(eloc, logpsi, weights=None):
    """(E complex, Var, sum of raw weights)."""
    lib = _load()
    e = np.ascontiguousarray(eloc, dtype=np.complex128)
    lp = np.ascontiguousarray(logpsi, dtype=np.complex128)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    st = np.empty(4)
    _check(lib.oracle_energy(e.size, _p(e), _p(lp), _p(w), _p(st)))
    return st[0] + 1j * st[1], st[2], st[3]


def adjoint(ham, keys, logpsi, eloc_rows, grad_e, weights=None, energy_value=None, rows=None):
    """Gradient of a real loss w.r.t. log psi for rows [a, b), given the
    upstream grad_e = dLoss/dRe E + i dLoss/dIm E."""
    lib = _load()
    c, xy, yz = _ham_arrays(ham)
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    lp = np.ascontiguousarray(logpsi, dtype=np.complex128)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    a, b = (0, keys.shape[0]) if rows is None else rows
    er = np.ascontiguousarray(eloc_rows, dtype=np.complex128)
    assert er.size == b - a
    en = None
    if weights is None:
        assert energy_value is not None, "|psi|^2 weights need E"
        en = np.array([energy_value.real, energy_value.imag])
    out = np.empty(b - a, dtype=np.complex128)
    _check(lib.oracle_adjoint(ham.n_qubits, ham.n_terms, _p(c), _p(xy), _p(yz), keys.shape[0],
                              _p(keys), _p(lp), _p(w), _p(er), _p(en),
                              float(np.real(grad_e)), float(np.imag(grad_e)), a, b, _p(out)))
    return out


MISS_TOL = 1e-10   # H_xx' counts as non-zero when |H_xx'| > MISS_TOL * sum |h_l| of its group


def find_misses(ham, keys, tol=MISS_TOL):
    """The states outside U coupled to U by a non-zero matrix element (the
    x' of Eq. local_energy that the sample-aware sum leaves out): uint64
    [n, W], unique, sorted ascending as W-word integers."""
    lib = _load()
    c, xy, yz = _ham_arrays(ham)
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    W = keys.shape[1]
    ptr = ctypes.POINTER(ctypes.c_uint64)()
    n = lib.oracle_find_misses(ham.n_qubits, ham.n_terms, _p(c), _p(xy), _p(yz), keys.shape[0], _p(keys),
                               float(tol), ctypes.byref(ptr))
    if n < 0:
        if ptr:
            lib.oracle_free(ptr)
        _check(int(n))
    try:
        out = np.ctypeslib.as_array(ptr, shape=(max(int(n), 1) * W,))[: int(n) * W].copy().reshape(int(n), W)
    finally:
        lib.oracle_free(ptr)
    return out


def local_energy_full(ham, keys, logpsi, keys_v, logpsi_v, tol=MISS_TOL, rows=None):
    """Conventional local energy (Eq. local_energy) for rows [a, b) of U,
    amplitudes of U from logpsi and of the extra states V from logpsi_v."""
    lib = _load()
    c, xy, yz = _ham_arrays(ham)
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    lp = np.ascontiguousarray(logpsi, dtype=np.complex128)
    kv = np.ascontiguousarray(keys_v, dtype=np.uint64).reshape(-1, keys.shape[1])
    lv = np.ascontiguousarray(logpsi_v, dtype=np.complex128)
    assert lv.size == kv.shape[0]
    a, b = (0, keys.shape[0]) if rows is None else rows
    out = np.empty(b - a, dtype=np.complex128)
    rc = lib.oracle_local_energy_full(ham.n_qubits, ham.n_terms, _p(c), _p(xy), _p(yz), keys.shape[0], _p(keys),
                                      _p(lp), kv.shape[0], _p(kv) if kv.size else None, _p(lv) if lv.size else None,
                                      float(tol), a, b, _p(out))
    if rc == -3:
        raise OracleError("a coupled state with a non-zero matrix element is in neither U nor V")
    _check(rc)
    return out
