"""Python binding of libeloc (the HIP engine for the sample-aware local
energy E_loc^var of arXiv 2408.07625).

Argument marshalling only: every step runs in the HIP kernels behind the C
ABI of include/eloc.h.  torch provides device memory and the stream.  There
is no CPU path: if libeloc.so has not been built, importing works but every
engine call raises.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

import numpy as np
import torch  # loads the HIP runtime that libeloc.so then binds to

_LIB_PATH = Path(__file__).resolve().parent / "libeloc.so"
_lib = None

VARIANTS = {"terms": 0, "batch": 1, "trie": 2, "auto": 3, "stored": 4}
PRECISIONS = {"fp64": 0, "fp32c": 1}
STATUS = {0: "OK", -1: "EINVAL", -2: "EDUP", -3: "ENOMEM", -4: "ECAPACITY", -5: "ERANGE", -6: "EHIP",
          -7: "ESTATE", -8: "EAGAIN"}
STATUS_CODE = {v: k for k, v in STATUS.items()}


class ElocError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class C64(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("chunks", ctypes.c_int), ("sig_filter", ctypes.c_int), ("rows_per_wave", ctypes.c_int),
                ("bloom", ctypes.c_int), ("waves_per_block", ctypes.c_int), ("partition", ctypes.c_int),
                ("partition_count", ctypes.c_int), ("trie_chunk", ctypes.c_int)]


class Problem(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int), ("n_terms", ctypes.c_int64), ("coeff", ctypes.c_void_p),
                ("xy", ctypes.c_void_p), ("yz", ctypes.c_void_p), ("n_unique", ctypes.c_int64),
                ("keys_dev", ctypes.c_void_p), ("logpsi_dev", ctypes.c_void_p), ("weights_dev", ctypes.c_void_p),
                ("eloc_dev", ctypes.c_void_p), ("stats_dev", ctypes.c_void_p)]


class ArModel(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int), ("qudit", ctypes.c_int), ("hidden", ctypes.c_int),
                ("n_up", ctypes.c_int), ("n_down", ctypes.c_int), ("W1", ctypes.c_void_p), ("b1", ctypes.c_void_p),
                ("W2", ctypes.c_void_p), ("b2", ctypes.c_void_p), ("W3", ctypes.c_void_p), ("b3", ctypes.c_void_p)]


class Schedule(ctypes.Structure):
    _fields_ = [("rows_per_wave", ctypes.c_int), ("blocks_per_cu", ctypes.c_int),
                ("item_candidates", ctypes.c_int64), ("order", ctypes.c_int), ("batch_ratio", ctypes.c_double)]


def library() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not _LIB_PATH.exists():
            raise RuntimeError(f"{_LIB_PATH} is not built; run python -m paper_2408_07625_amd.build")
        lib = ctypes.CDLL(str(_LIB_PATH))
        P, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
        sig = {
            "eloc_create": (i32, [ctypes.POINTER(P), i32, P]),
            "eloc_destroy": (None, [P]),
            "eloc_last_error": (ctypes.c_char_p, [P]),
            "eloc_set_stream": (i32, [P, P]),
            "eloc_set_hamiltonian": (i32, [P, i32, i64, P, P, P]),
            "eloc_hamiltonian_info": (i32, [P, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32)]),
            "eloc_set_samples": (i32, [P, i64, P]),
            "eloc_samples_info": (i32, [P, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32)]),
            "eloc_local_energy": (i32, [P, i32, i32, P, P, P, P]),
            "eloc_local_energy_noalloc": (i32, [P, i32, i32, P, P, P, P]),
            "eloc_find_misses": (i32, [P, ctypes.c_double, i64, P, ctypes.POINTER(i64)]),
            "eloc_local_energy_full": (i32, [P, i32, P, P, i64, P, P, P, P]),
            "eloc_sr_select": (i32, [P, i64, P, i32, P]),
            "eloc_sr_solve": (i32, [P, i32, i64, P, P, P, P, ctypes.c_double, P]),
            "eloc_sample": (i32, [P, ctypes.POINTER(ArModel), i64, ctypes.c_uint64, P, P, P, ctypes.POINTER(i64)]),
            "eloc_trie_visits": (i32, [P, ctypes.POINTER(i64)]),
            "eloc_check": (i32, [P]),
            "eloc_count_pairs": (i32, [P, i32, ctypes.POINTER(i64)]),
            "eloc_find_pairs": (i32, [P, i32, i64, P, P, P, ctypes.POINTER(i64)]),
            "eloc_pair_elements": (i32, [P, i64, P, P, P, P, P, i64]),
            "eloc_local_energy_adjoint": (i32, [P, i32, i32, P, P, P, P, C64, P]),
            "eloc_store_pairs": (i32, [P, i32, ctypes.c_size_t, ctypes.POINTER(i64)]),
            "eloc_set_tuning": (i32, [P, ctypes.POINTER(Tuning)]),
            "eloc_get_tuning": (i32, [P, ctypes.POINTER(Tuning)]),
            "eloc_profile_enable": (i32, [P, i32]),
            "eloc_profile_read": (i32, [P, P, P]),
            "eloc_batch_create": (i32, [ctypes.POINTER(P), i32, P, i32, P]),
            "eloc_batch_destroy": (None, [P]),
            "eloc_batch_last_error": (ctypes.c_char_p, [P]),
            "eloc_batch_set_stream": (i32, [P, P]),
            "eloc_batch_run": (i32, [P, i32]),
            "eloc_batch_set_graph": (i32, [P, i32]),
            "eloc_batch_check": (i32, [P, ctypes.POINTER(i32)]),
            "eloc_batch_pair_counts": (i32, [P, P]),
            "eloc_batch_problem_info": (i32, [P, i32, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                              ctypes.POINTER(i32), ctypes.POINTER(i32)]),
            "eloc_batch_get_schedule": (i32, [P, ctypes.POINTER(Schedule)]),
            "eloc_batch_set_schedule": (i32, [P, ctypes.POINTER(Schedule)]),
            "eloc_batch_tune": (i32, [P, i32, ctypes.c_char_p, ctypes.POINTER(i32)]),
            "eloc_batch_profile_enable": (i32, [P, i32]),
            "eloc_batch_profile_read": (i32, [P, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def exported_symbols() -> list[str]:
    """Names the header declares that the loaded library exports."""
    lib = library()
    return [n for n in ("eloc_create", "eloc_destroy", "eloc_last_error", "eloc_set_stream",
                        "eloc_set_hamiltonian", "eloc_hamiltonian_info", "eloc_set_samples", "eloc_samples_info",
                        "eloc_local_energy", "eloc_local_energy_noalloc", "eloc_find_misses",
                        "eloc_local_energy_full", "eloc_sr_select", "eloc_sr_solve", "eloc_sample", "eloc_trie_visits", "eloc_check", "eloc_count_pairs", "eloc_find_pairs",
                        "eloc_pair_elements", "eloc_local_energy_adjoint", "eloc_store_pairs", "eloc_set_tuning",
                        "eloc_get_tuning",
                        "eloc_profile_enable", "eloc_profile_read", "eloc_batch_create", "eloc_batch_destroy",
                        "eloc_batch_last_error", "eloc_batch_set_stream", "eloc_batch_run", "eloc_batch_set_graph",
                        "eloc_batch_check", "eloc_batch_pair_counts", "eloc_batch_problem_info",
                        "eloc_batch_get_schedule", "eloc_batch_set_schedule", "eloc_batch_tune",
                        "eloc_batch_profile_enable", "eloc_batch_profile_read")
            if hasattr(lib, n)]


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _np_ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _variant(v):
    return VARIANTS[v] if isinstance(v, str) else int(v)


def _precision(p):
    return PRECISIONS[p] if isinstance(p, str) else int(p)


class Engine:
    """One context of libeloc bound to a device and torch's current stream."""

    def __init__(self, device: int = 0):
        self.lib = library()
        self.device = torch.device("cuda", device)
        self.handle = ctypes.c_void_p()
        # without a visible GPU the library itself reports EINVAL
        stream = torch.cuda.current_stream(self.device).cuda_stream if torch.cuda.is_available() else 0
        self._call(self.lib.eloc_create(ctypes.byref(self.handle), device, ctypes.c_void_p(stream)))
        self.n_unique = 0
        self.n_qubits = 0
        # bumped by every call that changes the Hamiltonian, the samples or the
        # stored pair list: a backward pass refuses to run on other state than
        # its forward pass saw
        self.generation = 0

    def close(self):
        if self.handle:
            self.lib.eloc_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, rc):
        if rc != 0:
            msg = self.lib.eloc_last_error(self.handle) if self.handle else b""
            raise ElocError(rc, (msg or b"").decode())
        return rc

    def _sync_stream(self):
        self._call(self.lib.eloc_set_stream(self.handle,
                                            ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)))

    # -- inputs -------------------------------------------------------------
    def set_hamiltonian(self, n_qubits: int, coeff, xy, yz):
        c = np.ascontiguousarray(coeff, dtype=np.float64)
        xy = np.ascontiguousarray(xy, dtype=np.uint64)
        yz = np.ascontiguousarray(yz, dtype=np.uint64)
        W = (n_qubits + 63) // 64
        assert xy.shape == (c.size, W) and yz.shape == (c.size, W)
        self._sync_stream()
        self.generation += 1
        self._call(self.lib.eloc_set_hamiltonian(self.handle, n_qubits, c.size, _np_ptr(c), _np_ptr(xy),
                                                 _np_ptr(yz)))
        self.n_qubits = n_qubits
        self.n_unique = 0

    def info(self):
        g, t, n = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int()
        self._call(self.lib.eloc_hamiltonian_info(self.handle, ctypes.byref(g), ctypes.byref(t), ctypes.byref(n)))
        return {"n_groups": g.value, "n_terms": t.value, "n_qubits": n.value}

    def set_samples(self, keys: torch.Tensor, check: bool = True):
        """keys: int64/uint64 device tensor [M, W] (bit patterns).  The
        library prepares U asynchronously; with check (default) this waits
        and raises EDUP / EINVAL for invalid samples, else they are reported
        by the next check()."""
        W = (self.n_qubits + 63) // 64
        if not (keys.is_cuda and keys.dtype in (torch.int64, torch.uint64) and keys.is_contiguous()
                and keys.dim() == 2 and keys.shape[1] == W):
            raise ValueError(f"keys must be a contiguous int64 CUDA tensor [M, {W}]")
        self.generation += 1
        self._sync_stream()
        self._call(self.lib.eloc_set_samples(self.handle, keys.shape[0], _ptr(keys)))
        self.n_unique = keys.shape[0]
        if check:
            self.check()

    def samples_info(self) -> dict:
        """Size of U and of its membership table (slots, keys in the stash)."""
        n, slots, stash = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        self._call(self.lib.eloc_samples_info(self.handle, ctypes.byref(n), ctypes.byref(slots), ctypes.byref(stash)))
        return {"n_unique": n.value, "table_slots": slots.value, "table_stash": stash.value}

    def set_tuning(self, chunks: int = 0, sig_filter: bool = True, rows_per_wave: int = 0, bloom: bool = False,
                   waves_per_block: int = 0, partition: int = 0, partition_count: int = 0, trie_chunk: int = 0):
        """partition: 0 automatic (U tables of 8 MB and more), 1 on, -1 off;
        partition_count: 8, 16 or 32 (0 automatic).  Set before
        set_hamiltonian and set_samples (the group records are bucketed at
        ingest, U's rows classed when its table is built).  trie_chunk: XY
        masks per LoopOverTrie chunk tree (0 automatic; used from the next
        set_samples)."""
        t = Tuning(int(chunks), 1 if sig_filter else 0, int(rows_per_wave), 1 if bloom else 0, int(waves_per_block),
                   int(partition), int(partition_count), int(trie_chunk))
        self._call(self.lib.eloc_set_tuning(self.handle, ctypes.byref(t)))

    def get_tuning(self) -> dict:
        t = Tuning()
        self._call(self.lib.eloc_get_tuning(self.handle, ctypes.byref(t)))
        return {"chunks": t.chunks, "sig_filter": bool(t.sig_filter), "rows_per_wave": t.rows_per_wave,
                "bloom": bool(t.bloom), "waves_per_block": t.waves_per_block, "partition": t.partition,
                "partition_count": t.partition_count, "trie_chunk": t.trie_chunk}

    STAGES = ("samples", "amplitudes", "pairs", "finish", "energy", "adjoint_pairs", "adjoint_finish")

    def profile(self, on: bool = True):
        self._call(self.lib.eloc_profile_enable(self.handle, 1 if on else 0))

    def profile_read(self) -> dict:
        """{stage: (total ms, launches)} since the last read (synchronises)."""
        ms = np.zeros(len(self.STAGES), dtype=np.float64)
        cnt = np.zeros(len(self.STAGES), dtype=np.int64)
        self._call(self.lib.eloc_profile_read(self.handle, _np_ptr(ms), _np_ptr(cnt)))
        return {s: (float(ms[k]), int(cnt[k])) for k, s in enumerate(self.STAGES)}

    # -- forward ------------------------------------------------------------
    def local_energy(self, logpsi: torch.Tensor, weights: torch.Tensor | None = None, variant="terms",
                     precision="fp64", out: torch.Tensor | None = None, stats: torch.Tensor | None = None,
                     check: bool = True):
        """Returns (E_loc complex128 [M], stats float64 [4] = Re E, Im E, Var, sum w)."""
        M = self.n_unique if self.n_unique else logpsi.shape[0]   # no batch yet: the library says ESTATE
        if logpsi.dtype != torch.complex128 or not logpsi.is_cuda or logpsi.shape != (M,):
            raise ValueError("logpsi must be a complex128 CUDA tensor with one entry per sample")
        logpsi = logpsi.contiguous()
        if weights is not None:
            if weights.dtype != torch.float64 or not weights.is_cuda or weights.shape != (M,):
                raise ValueError("weights must be a float64 CUDA tensor with one entry per sample")
            weights = weights.contiguous()
        if out is None:
            out = torch.empty(M, dtype=torch.complex128, device=self.device)
        if stats is None:
            stats = torch.empty(4, dtype=torch.float64, device=self.device)
        self._sync_stream()
        self._call(self.lib.eloc_local_energy(self.handle, _variant(variant), _precision(precision), _ptr(logpsi),
                                              _ptr(weights), _ptr(out), _ptr(stats)))
        if check:
            self.check()
        return out, stats

    def check(self):
        self._call(self.lib.eloc_check(self.handle))

    # -- sampling without replacement ----------------------------------------
    def sample(self, n_qubits: int, qudit: int, weights: dict, k: int, seed: int, n_up: int = -1,
               n_down: int = -1):
        """ARGumbelTopK over the per-qudit perceptron ansatz.  weights: float64
        CUDA tensors W1 [Q,64,N], b1 [Q,64], W2 [Q,64,64], b2 [Q,64], W3
        [Q,2^qudit,64], b3 [Q,2^qudit].  Returns (keys int64 [n, W], log p
        float64 [n], perturbed log-probabilities float64 [n]), n <= k."""
        Q = (n_qubits + qudit - 1) // qudit
        shapes = {"W1": (Q, 64, n_qubits), "b1": (Q, 64), "W2": (Q, 64, 64), "b2": (Q, 64),
                  "W3": (Q, 1 << qudit, 64), "b3": (Q, 1 << qudit)}
        ws = {}
        for name, shape in shapes.items():
            t = weights[name]
            if t.dtype != torch.float64 or not t.is_cuda or tuple(t.shape) != shape:
                raise ValueError(f"{name} must be a float64 CUDA tensor of shape {shape}")
            ws[name] = t.contiguous()
        m = ArModel(int(n_qubits), int(qudit), 64, int(n_up), int(n_down), *(ws[n].data_ptr() for n in
                                                                          ("W1", "b1", "W2", "b2", "W3", "b3")))
        W = (n_qubits + 63) // 64
        keys = torch.empty((k, W), dtype=torch.int64, device=self.device)
        logp = torch.empty(k, dtype=torch.float64, device=self.device)
        pert = torch.empty(k, dtype=torch.float64, device=self.device)
        n = ctypes.c_int64()
        self._sync_stream()
        self._call(self.lib.eloc_sample(self.handle, ctypes.byref(m), int(k), ctypes.c_uint64(seed & ((1 << 64) - 1)),
                                        _ptr(keys), _ptr(logp), _ptr(pert), ctypes.byref(n)))
        return keys[: n.value], logp[: n.value], pert[: n.value]

    # -- stochastic reconfiguration ------------------------------------------
    def sr_select(self, logpsi: torch.Tensor, n_sr: int) -> torch.Tensor:
        """Indices (int32 [n_sr]) of the n_sr largest Re log psi, descending."""
        if logpsi.dtype != torch.complex128 or not logpsi.is_cuda or logpsi.dim() != 1:
            raise ValueError("logpsi must be a complex128 CUDA vector")
        logpsi = logpsi.contiguous()
        out = torch.empty(n_sr, dtype=torch.int32, device=self.device)
        self._sync_stream()
        self._call(self.lib.eloc_sr_select(self.handle, logpsi.shape[0], _ptr(logpsi), int(n_sr), _ptr(out)))
        return out

    def sr_solve(self, o_re: torch.Tensor, o_im: torch.Tensor, logpsi_set: torch.Tensor, grad: torch.Tensor,
                 lam: float, out: torch.Tensor | None = None, check: bool = True) -> torch.Tensor:
        """(Re S + lam I)^{-1} grad with S estimated over the set (float64 [n_params])."""
        n_sr, n_p = o_re.shape
        for t, name in ((o_re, "o_re"), (o_im, "o_im")):
            if t.dtype != torch.float64 or not t.is_cuda or tuple(t.shape) != (n_sr, n_p):
                raise ValueError(f"{name} must be a float64 CUDA tensor [n_sr, n_params]")
        if logpsi_set.dtype != torch.complex128 or not logpsi_set.is_cuda or logpsi_set.shape != (n_sr,):
            raise ValueError("logpsi_set must be a complex128 CUDA tensor [n_sr]")
        if grad.dtype != torch.float64 or not grad.is_cuda or grad.shape != (n_p,):
            raise ValueError("grad must be a float64 CUDA tensor [n_params]")
        o_re, o_im, logpsi_set, grad = o_re.contiguous(), o_im.contiguous(), logpsi_set.contiguous(), grad.contiguous()
        if out is None:
            out = torch.empty(n_p, dtype=torch.float64, device=self.device)
        self._sync_stream()
        self._call(self.lib.eloc_sr_solve(self.handle, n_sr, n_p, _ptr(o_re), _ptr(o_im), _ptr(logpsi_set),
                                          _ptr(grad), float(lam), _ptr(out)))
        if check:
            self.check()
        return out

    # -- conventional local energy -------------------------------------------
    def find_misses(self, tol: float = 1e-10) -> torch.Tensor:
        """States outside U coupled to U by a non-zero matrix element: int64
        device tensor [n, W] (bit patterns), sorted, each once."""
        n = ctypes.c_int64()
        self._sync_stream()
        rc = self.lib.eloc_find_misses(self.handle, float(tol), 0, None, ctypes.byref(n))
        if rc != STATUS_CODE["ECAPACITY"]:   # the count comes back with ECAPACITY unless it is 0
            self._call(rc)
        W = (self.n_qubits + 63) // 64
        out = torch.empty((max(n.value, 1), W), dtype=torch.int64, device=self.device)
        self._call(self.lib.eloc_find_misses(self.handle, float(tol), n.value, _ptr(out), ctypes.byref(n)))
        return out[: n.value]

    def local_energy_full(self, logpsi: torch.Tensor, extra_keys: torch.Tensor, extra_logpsi: torch.Tensor,
                          weights: torch.Tensor | None = None, precision="fp64"):
        """Conventional local energy of every sample (Eq. local_energy): (E_loc
        complex128 [M], stats float64 [4]) from U's and the extra states'
        log-amplitudes."""
        M = self.n_unique
        W = (self.n_qubits + 63) // 64
        if logpsi.dtype != torch.complex128 or not logpsi.is_cuda or logpsi.shape != (M,):
            raise ValueError("logpsi must be a complex128 CUDA tensor with one entry per sample")
        n = extra_keys.shape[0]
        if not (extra_keys.is_cuda and extra_keys.dtype in (torch.int64, torch.uint64) and extra_keys.dim() == 2
                and extra_keys.shape[1] == W):
            raise ValueError(f"extra_keys must be an int64 CUDA tensor [n, {W}]")
        if extra_logpsi.dtype != torch.complex128 or not extra_logpsi.is_cuda or extra_logpsi.shape != (n,):
            raise ValueError("extra_logpsi must be a complex128 CUDA tensor [n]")
        if weights is not None and (weights.dtype != torch.float64 or not weights.is_cuda or weights.shape != (M,)):
            raise ValueError("weights must be a float64 CUDA tensor with one entry per sample")
        logpsi, extra_keys, extra_logpsi = logpsi.contiguous(), extra_keys.contiguous(), extra_logpsi.contiguous()
        weights = None if weights is None else weights.contiguous()
        out = torch.empty(M, dtype=torch.complex128, device=self.device)
        stats = torch.empty(4, dtype=torch.float64, device=self.device)
        self._sync_stream()
        self._call(self.lib.eloc_local_energy_full(self.handle, _precision(precision), _ptr(logpsi), _ptr(weights),
                                                   n, _ptr(extra_keys) if n else None,
                                                   _ptr(extra_logpsi) if n else None, _ptr(out), _ptr(stats)))
        return out, stats

    # -- pairs --------------------------------------------------------------
    def count_pairs(self, variant="terms") -> int:
        n = ctypes.c_int64()
        self._sync_stream()
        self._call(self.lib.eloc_count_pairs(self.handle, _variant(variant), ctypes.byref(n)))
        return n.value

    def trie_visits(self) -> int:
        """Node pairs LoopOverTrie's walk visits for the current samples."""
        n = ctypes.c_int64()
        self._sync_stream()
        self._call(self.lib.eloc_trie_visits(self.handle, ctypes.byref(n)))
        return n.value

    def find_pairs(self, variant="terms"):
        """Canonical coupled pairs (i, j, g) sorted by (i, j), int32 device tensors."""
        n = self.count_pairs(variant)
        cap = max(n, 1)
        i = torch.empty(cap, dtype=torch.int32, device=self.device)
        j = torch.empty(cap, dtype=torch.int32, device=self.device)
        g = torch.empty(cap, dtype=torch.int32, device=self.device)
        got = ctypes.c_int64()
        self._call(self.lib.eloc_find_pairs(self.handle, _variant(variant), cap, _ptr(i), _ptr(j), _ptr(g),
                                            ctypes.byref(got)))
        k = got.value
        return i[:k], j[:k], g[:k]

    def store_pairs(self, variant="auto", budget_bytes: int | None = None) -> int:
        """Keep the pair list of the current samples for variant "stored";
        returns the pair count.  ElocError ECAPACITY if it needs more than
        budget_bytes (default: half of the free device memory)."""
        if budget_bytes is None:
            budget_bytes = torch.cuda.mem_get_info(self.device)[0] // 2
        n = ctypes.c_int64()
        self.generation += 1
        self._sync_stream()
        self._call(self.lib.eloc_store_pairs(self.handle, _variant(variant), int(budget_bytes), ctypes.byref(n)))
        return n.value

    def pair_elements(self, i: torch.Tensor, j: torch.Tensor, phases: bool = False):
        """H_{x_i x_j} (complex128 [n]); with phases also (term_offsets int64
        [n + 1], k uint8 [term_offsets[n]]): the exponent k of i^k of every
        term of the pair's group, terms in ascending caller index."""
        if not (i.dtype == torch.int32 and j.dtype == torch.int32 and i.shape == j.shape and i.dim() == 1
                and i.is_cuda and j.is_cuda):
            raise ValueError("i and j must be int32 CUDA tensors of one shape [n]")
        i, j = i.contiguous(), j.contiguous()
        n = i.shape[0]
        h = torch.empty(n, dtype=torch.complex128, device=self.device)
        self._sync_stream()
        if not phases:
            self._call(self.lib.eloc_pair_elements(self.handle, n, _ptr(i), _ptr(j), _ptr(h), None, None, 0))
            self.check()
            return h
        off = torch.empty(n + 1, dtype=torch.int64, device=self.device)
        self._call(self.lib.eloc_pair_elements(self.handle, n, _ptr(i), _ptr(j), _ptr(h), _ptr(off), None, 0))
        self.check()
        total = int(off[n].item())
        k = torch.empty(max(total, 1), dtype=torch.uint8, device=self.device)
        self._call(self.lib.eloc_pair_elements(self.handle, n, _ptr(i), _ptr(j), _ptr(h), _ptr(off), _ptr(k),
                                               total))
        self.check()
        return h, off, k[:total]

    # -- adjoint ------------------------------------------------------------
    def adjoint(self, logpsi, eloc, stats, grad_e: complex, weights=None, variant="terms", precision="fp64",
                out=None, check=True):
        """dLoss/dlog psi [M] (complex128) for upstream grad_e = dLoss/dRe E +
        i dLoss/dIm E; eloc and stats are the forward outputs for the same
        logpsi and weights."""
        M = self.n_unique

        def need(t, name, dtype, shape):
            if t is None or t.dtype != dtype or not t.is_cuda or tuple(t.shape) != shape:
                raise ValueError(f"{name} must be a {dtype} CUDA tensor of shape {shape}")
            return t.contiguous()

        logpsi = need(logpsi, "logpsi", torch.complex128, (M,))
        eloc = need(eloc, "eloc", torch.complex128, (M,))
        stats = need(stats, "stats", torch.float64, (4,))
        if weights is not None:
            weights = need(weights, "weights", torch.float64, (M,))
        if out is None:
            out = torch.empty(M, dtype=torch.complex128, device=self.device)
        else:
            need(out, "out", torch.complex128, (M,))
            if not out.is_contiguous():
                raise ValueError("out must be contiguous")
        ge = C64(float(np.real(grad_e)), float(np.imag(grad_e)))
        self._sync_stream()
        self._call(self.lib.eloc_local_energy_adjoint(self.handle, _variant(variant), _precision(precision),
                                                      _ptr(logpsi), _ptr(weights), _ptr(eloc), _ptr(stats), ge,
                                                      _ptr(out)))
        if check:
            self.check()
        return out


class LocalEnergy(torch.autograd.Function):
    """E = sum_x w~_x E_loc^var(x) as a differentiable function of log psi.

    forward(logpsi, weights, engine, variant, precision, store_budget) ->
    (E complex128 scalar, E_loc [M] (not differentiable), stats [4]).
    Backward calls the adjoint kernels.  With store_budget (bytes) the pair
    list is stored when it fits and both passes read it; otherwise the
    backward finds the pairs again."""

    @staticmethod
    def forward(ctx, logpsi, weights, engine, variant="terms", precision="fp64", store_budget=None):
        if store_budget is not None:
            try:
                engine.store_pairs(variant, store_budget)
                variant = "stored"
            except ElocError as e:
                if e.status != "ECAPACITY":
                    raise
        eloc, stats = engine.local_energy(logpsi, weights, variant, precision)
        ctx.engine, ctx.variant, ctx.precision = engine, variant, precision
        ctx.generation = engine.generation
        ctx.save_for_backward(logpsi, eloc, stats, *( [weights] if weights is not None else []))
        ctx.has_w = weights is not None
        E = torch.complex(stats[0], stats[1])
        ctx.mark_non_differentiable(eloc, stats)
        return E, eloc, stats

    @staticmethod
    def backward(ctx, grad_E, grad_eloc, grad_stats):
        saved = ctx.saved_tensors
        logpsi, eloc, stats = saved[:3]
        weights = saved[3] if ctx.has_w else None
        if ctx.engine.generation != ctx.generation:
            raise RuntimeError("the engine's Hamiltonian, samples or stored pairs changed between the forward "
                               "and the backward pass of LocalEnergy")
        ge = complex(grad_E.item()) if grad_E is not None else 0j
        g = ctx.engine.adjoint(logpsi, eloc, stats, ge, weights, ctx.variant, ctx.precision)
        return g, None, None, None, None, None


def local_energy(engine: Engine, logpsi, weights=None, variant="terms", precision="fp64", store_budget=None):
    return LocalEnergy.apply(logpsi, weights, engine, variant, precision, store_budget)


class Batch:
    """Many (Hamiltonian, U) problems evaluated by one batched launch.

    problems: sequence of dicts with n_qubits, coeff, xy, yz (host arrays as
    for Engine.set_hamiltonian), keys (int64 device tensor [M, W_k]), logpsi
    (complex128 device tensor [M]) and optionally weights (float64 device
    tensor [M]).  The device tensors are kept referenced: every run reads
    their current contents, so new samples of the same sizes are passed by
    writing into them (self.inputs[k]).  Outputs: self.eloc[k] (complex128
    [M_k]) and self.stats[k] (float64 [4]) per problem."""

    def __init__(self, problems, device: int = 0):
        self.lib = library()
        self.device = torch.device("cuda", device)
        self.handle = ctypes.c_void_p()
        self._host = []
        self.inputs, self.eloc, self.stats = [], [], []
        arr = (Problem * len(problems))()
        for k, p in enumerate(problems):
            c = np.ascontiguousarray(p["coeff"], dtype=np.float64)
            xy = np.ascontiguousarray(p["xy"], dtype=np.uint64)
            yz = np.ascontiguousarray(p["yz"], dtype=np.uint64)
            keys = p["keys"]
            if not (keys.is_cuda and keys.dtype in (torch.int64, torch.uint64) and keys.is_contiguous()):
                raise ValueError(f"problem {k}: keys must be a contiguous int64 CUDA tensor")
            lp = p["logpsi"]
            if lp.dtype != torch.complex128 or not lp.is_cuda or lp.shape != (keys.shape[0],) or \
                    not lp.is_contiguous():
                raise ValueError(f"problem {k}: logpsi must be a contiguous complex128 CUDA tensor [M]")
            w = p.get("weights")
            if w is not None and (w.dtype != torch.float64 or not w.is_cuda or w.shape != (keys.shape[0],) or
                                  not w.is_contiguous()):
                raise ValueError(f"problem {k}: weights must be a contiguous float64 CUDA tensor [M]")
            e = torch.empty(keys.shape[0], dtype=torch.complex128, device=self.device)
            s = torch.empty(4, dtype=torch.float64, device=self.device)
            self.eloc.append(e)
            self.stats.append(s)
            self._host += [c, xy, yz]
            self.inputs.append({"keys": keys, "logpsi": lp, "weights": w})
            arr[k] = Problem(int(p["n_qubits"]), c.size, _np_ptr(c).value, _np_ptr(xy).value, _np_ptr(yz).value,
                             keys.shape[0], keys.data_ptr(), lp.data_ptr(), None if w is None else w.data_ptr(),
                             e.data_ptr(), s.data_ptr())
        stream = torch.cuda.current_stream(self.device).cuda_stream if torch.cuda.is_available() else 0
        rc = self.lib.eloc_batch_create(ctypes.byref(self.handle), device, ctypes.c_void_p(stream), len(problems),
                                        ctypes.cast(arr, ctypes.c_void_p))
        self._call(rc)
        self.n = len(problems)
        self._host = []   # copied by create; the device tensors in self.inputs must live on

    def close(self):
        if self.handle:
            self.lib.eloc_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, rc, bad=None):
        if rc != 0:
            msg = (self.lib.eloc_batch_last_error(self.handle) or b"").decode() if self.handle else ""
            err = ElocError(rc, msg)
            err.problem = None if bad is None else bad.value
            raise err
        return rc

    def _sync_stream(self):
        self._call(self.lib.eloc_batch_set_stream(
            self.handle, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)))

    def run(self, precision="fp32c", check: bool = True):
        self._sync_stream()
        self._call(self.lib.eloc_batch_run(self.handle, _precision(precision)))
        if check:
            self.check()
        return self.eloc, self.stats

    def check(self):
        bad = ctypes.c_int(-1)
        self._call(self.lib.eloc_batch_check(self.handle, ctypes.byref(bad)), bad)

    def set_graph(self, on: bool):
        self._call(self.lib.eloc_batch_set_graph(self.handle, 1 if on else 0))

    def profile(self, on: bool):
        """Stage timing of eager runs (set_graph(False)) with HIP events."""
        self._call(self.lib.eloc_batch_profile_enable(self.handle, 1 if on else 0))

    def profile_read(self) -> dict:
        """{stage: (total ms, runs)} since the last read, stages prepare,
        pairs, finish; synchronising."""
        ms = np.zeros(3, dtype=np.float64)
        n = np.zeros(3, dtype=np.int64)
        self._call(self.lib.eloc_batch_profile_read(self.handle, _np_ptr(ms), _np_ptr(n)))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(("prepare", "pairs", "finish"))}

    def pair_counts(self) -> np.ndarray:
        out = np.zeros(self.n, dtype=np.int64)
        self._call(self.lib.eloc_batch_pair_counts(self.handle, _np_ptr(out)))
        return out

    def problem_info(self, k: int) -> dict:
        g, t, v, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int(), ctypes.c_int()
        self._call(self.lib.eloc_batch_problem_info(self.handle, k, ctypes.byref(g), ctypes.byref(t),
                                                    ctypes.byref(v), ctypes.byref(c)))
        return {"n_groups": g.value, "n_terms": t.value, "variant": "batch" if v.value == 1 else "terms",
                "chunks": c.value}

    def get_schedule(self) -> dict:
        s = Schedule()
        self._call(self.lib.eloc_batch_get_schedule(self.handle, ctypes.byref(s)))
        return {"rows_per_wave": s.rows_per_wave, "blocks_per_cu": s.blocks_per_cu,
                "item_candidates": s.item_candidates, "order": s.order, "batch_ratio": s.batch_ratio}

    def set_schedule(self, rows_per_wave=8, blocks_per_cu=0, item_candidates=1 << 17, order=0, batch_ratio=1.0):
        s = Schedule(int(rows_per_wave), int(blocks_per_cu), int(item_candidates), int(order), float(batch_ratio))
        self._call(self.lib.eloc_batch_set_schedule(self.handle, ctypes.byref(s)))

    def tune(self, precision="fp32c", cache_path=None) -> tuple[dict, bool]:
        """Autotune the schedule (synchronising); returns (schedule, taken from the cache)."""
        self._sync_stream()
        hit = ctypes.c_int(0)
        path = None if cache_path is None else str(cache_path).encode()
        self._call(self.lib.eloc_batch_tune(self.handle, _precision(precision), path, ctypes.byref(hit)))
        return self.get_schedule(), bool(hit.value)
