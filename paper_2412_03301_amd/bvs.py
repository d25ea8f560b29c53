"""ctypes binding of libbvs.so (the C ABI in include/bvs.h).

Argument marshalling only: every step of the search runs in the HIP
library.  PyTorch supplies device memory (index, workspaces, outputs) and
the current stream.  Importing torch before loading the library makes the
library share torch's HIP runtime.  There is no fallback: if the library
is not built, `lib()` raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbvs.so")

BVS_OK, BVS_EINVAL, BVS_ERANGE, BVS_ENOSPC, BVS_EDEVICE, BVS_ESTATE, BVS_ENOTSUP = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ERANGE", -3: "ENOSPC", -4: "EDEVICE", -5: "ESTATE", -6: "ENOTSUP"}

EXPORTED = [
    "bvs_params_default", "bvs_params_check", "bvs_projection", "bvs_index_bytes",
    "bvs_build_workspace_bytes", "bvs_build_index", "bvs_index_destroy", "bvs_index_get_info",
    "bvs_index_get_params", "bvs_sketch_views", "bvs_encode_workspace_bytes", "bvs_encode",
    "bvs_search_workspace_bytes", "bvs_query_sketch", "bvs_search_candidates", "bvs_search",
    "bvs_bruteforce_workspace_bytes", "bvs_bruteforce", "bvs_hausdorff_all", "bvs_last_error",
    "bvs_version", "bvs_profile_enable", "bvs_profile_read", "bvs_stage_name",
    "bvs_batch_create", "bvs_batch_bind", "bvs_batch_launch", "bvs_batch_status", "bvs_batch_get_info",
    "bvs_batch_destroy", "bvs_lowp_bytes", "bvs_lowp_attach", "bvs_lowp_workspace_bytes", "bvs_search_lowp",
    "bvs_hausdorff_lowp", "bvs_mlp_weight_count", "bvs_mlp_init", "bvs_learned_index_bytes",
    "bvs_learned_build_workspace_bytes", "bvs_build_index_learned", "bvs_train_workspace_bytes",
    "bvs_train_gradients", "bvs_train_projection", "bvs_search_noalloc_max_bytes", "bvs_search_noalloc",
    "bvs_search_metric", "bvs_bruteforce_metric", "bvs_codes_bytes", "bvs_codes_attach_workspace_bytes",
    "bvs_codes_attach", "bvs_search_full_workspace_bytes", "bvs_full_scores", "bvs_search_full_candidates",
    "bvs_search_full", "bvs_index_set_search_params", "bvs_lists_workspace_bytes", "bvs_lists_bytes",
    "bvs_lists_attach", "bvs_lists_views", "bvs_index_set_first_layer", "bvs_train_state_bytes",
    "bvs_train_state_init", "bvs_train_projection_resume",
]
FIRST_LAYER = {"bitmaps": 0, "lists": 1}
METRIC = {"hausdorff": 0, "meanmin": 1, "min": 2}
LOWP = {"bf16": 1, "fp8": 2}
TUNE_MAX = 16
BVS_BATCH_PHASES = 1   # bvs_batch_config.flags: the phase sequence by size class
N_STAGES = 14
N_COUNTERS = 7
COUNTER_NAMES = ("filter_pairs", "rerank_vectors", "rerank_abandoned", "rerank_candidates",
                 "rerank_screen_vectors", "rerank_screened", "lowp_vectors")


class Params(C.Structure):
    _fields_ = [("dim", C.c_uint32), ("code_bits", C.c_uint32), ("fan_in", C.c_uint32),
                ("wta_k", C.c_uint32), ("access_lists", C.c_uint32), ("min_count", C.c_uint32),
                ("top_t", C.c_uint32), ("flags", C.c_uint32), ("seed", C.c_uint64)]

    @classmethod
    def make(cls, dim, code_bits=1024, fan_in=8, wta_k=64, access_lists=3, min_count=1,
             top_t=1000, seed=0):
        return cls(dim, code_bits, fan_in, wta_k, access_lists, min_count, top_t, 0, seed)


class IndexInfo(C.Structure):
    _fields_ = [("n_sets", C.c_uint64), ("n_vectors", C.c_uint64), ("ld_sets", C.c_uint64),
                ("dim_padded", C.c_uint32), ("max_set_size", C.c_uint32)]


class StageTimes(C.Structure):
    _fields_ = [("ms", C.c_double * N_STAGES), ("calls", C.c_uint64 * N_STAGES),
                ("counters", C.c_uint64 * N_COUNTERS)]


class BatchConfig(C.Structure):
    _fields_ = [("lds_rows", C.c_uint32), ("waves", C.c_uint32), ("graph", C.c_uint32), ("flags", C.c_uint32)]


class BatchInfo(C.Structure):
    _fields_ = [("n_q", C.c_uint32), ("max_rows", C.c_uint32), ("n_q_vectors", C.c_uint64),
                ("workspace_bytes", C.c_uint64), ("lds_rows", C.c_uint32), ("waves", C.c_uint32),
                ("blocks", C.c_uint32), ("from_cache", C.c_uint32), ("graph", C.c_uint32),
                ("n_tried", C.c_uint32), ("tried_lds_rows", C.c_uint32 * TUNE_MAX),
                ("tried_waves", C.c_uint32 * TUNE_MAX), ("tried_ms", C.c_float * TUNE_MAX)]


class TrainConfig(C.Structure):
    _fields_ = [("dim", C.c_uint32), ("hidden", C.c_uint32), ("code_bits", C.c_uint32), ("wta_k", C.c_uint32),
                ("batch_triplets", C.c_uint32), ("epochs", C.c_uint32), ("lr", C.c_float), ("tau", C.c_float),
                ("margin", C.c_float), ("reserved", C.c_uint32), ("seed", C.c_uint64)]


class BvsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None
P = C.c_void_p
U32, U64 = C.c_uint32, C.c_uint64
PU64 = C.POINTER(C.c_uint64)


def lib():
    """Load libbvs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; build it with "
                               "python -m paper_2412_03301_amd.csrc.build")
        L = C.CDLL(LIB_PATH)
        sig = {
            "bvs_params_default": (None, [P]),
            "bvs_params_check": (C.c_int, [P]),
            "bvs_projection": (C.c_int, [P, P]),
            "bvs_index_bytes": (C.c_int, [P, U64, U64, PU64]),
            "bvs_build_workspace_bytes": (C.c_int, [P, U64, U64, PU64]),
            "bvs_build_index": (C.c_int, [P, P, P, U64, P, U64, P, U64, P, C.POINTER(P)]),
            "bvs_index_destroy": (None, [P]),
            "bvs_index_get_info": (C.c_int, [P, P]),
            "bvs_index_get_params": (C.c_int, [P, P]),
            "bvs_sketch_views": (C.c_int, [P, C.POINTER(P), C.POINTER(P)]),
            "bvs_encode_workspace_bytes": (C.c_int, [P, U64, PU64]),
            "bvs_encode": (C.c_int, [P, P, U64, P, U64, P, P]),
            "bvs_search_workspace_bytes": (C.c_int, [P, U32, U64, PU64]),
            "bvs_query_sketch": (C.c_int, [P, P, P, U32, P, U64, P, P, P, P]),
            "bvs_search_candidates": (C.c_int, [P, P, P, U32, P, U64, P, P, P, P]),
            "bvs_search": (C.c_int, [P, P, P, U32, U32, P, U64, P, P, P, P]),
            "bvs_search_noalloc_max_bytes": (U64, []),
            "bvs_search_metric": (C.c_int, [P, C.c_int, P, P, U32, U32, P, U64, P, P, P, P]),
            "bvs_bruteforce_metric": (C.c_int, [P, C.c_int, P, P, U32, U32, P, U64, P, P, P, P]),
            "bvs_search_noalloc": (C.c_int, [P, P, P, U32, U32, P, P, P, P]),
            "bvs_index_set_search_params": (C.c_int, [P, U32, U32, U32]),
            "bvs_lists_workspace_bytes": (C.c_int, [P, PU64]),
            "bvs_lists_bytes": (C.c_int, [P, P, U64, P, PU64]),
            "bvs_lists_attach": (C.c_int, [P, P, U64, P, U64, P]),
            "bvs_lists_views": (C.c_int, [P, C.POINTER(P), C.POINTER(P), C.POINTER(P), PU64]),
            "bvs_index_set_first_layer": (C.c_int, [P, C.c_int]),
            "bvs_codes_bytes": (C.c_int, [P, PU64]),
            "bvs_codes_attach_workspace_bytes": (C.c_int, [P, PU64]),
            "bvs_codes_attach": (C.c_int, [P, P, U64, P, U64, P]),
            "bvs_search_full_workspace_bytes": (C.c_int, [P, U32, U64, PU64]),
            "bvs_full_scores": (C.c_int, [P, P, P, U32, P, U64, P, P]),
            "bvs_search_full_candidates": (C.c_int, [P, P, P, U32, P, U64, P, P, P, P]),
            "bvs_search_full": (C.c_int, [P, P, P, U32, U32, P, U64, P, P, P, P]),
            "bvs_bruteforce_workspace_bytes": (C.c_int, [P, U32, U64, PU64]),
            "bvs_bruteforce": (C.c_int, [P, P, P, U32, U32, P, U64, P, P, P, P]),
            "bvs_hausdorff_all": (C.c_int, [P, P, P, U32, P, U64, P, P]),
            "bvs_last_error": (C.c_char_p, []),
            "bvs_version": (C.c_char_p, []),
            "bvs_profile_enable": (C.c_int, [C.c_int]),
            "bvs_profile_read": (C.c_int, [P]),
            "bvs_stage_name": (C.c_char_p, [C.c_int]),
            "bvs_batch_create": (C.c_int, [P, P, U32, U32, P, C.POINTER(P)]),
            "bvs_batch_bind": (C.c_int, [P, P, P, U64, P, P, P, P]),
            "bvs_batch_launch": (C.c_int, [P, P]),
            "bvs_batch_status": (C.c_int, [P, P]),
            "bvs_batch_get_info": (C.c_int, [P, P]),
            "bvs_batch_destroy": (None, [P]),
            "bvs_lowp_bytes": (C.c_int, [P, C.c_int, PU64]),
            "bvs_lowp_attach": (C.c_int, [P, C.c_int, P, U64, P]),
            "bvs_lowp_workspace_bytes": (C.c_int, [P, U32, U64, PU64]),
            "bvs_search_lowp": (C.c_int, [P, C.c_int, C.c_float, P, P, U32, U32, P, U64, P, P, P, P, P]),
            "bvs_hausdorff_lowp": (C.c_int, [P, C.c_int, P, P, U32, P, U32, P, U64, P, P]),
            "bvs_mlp_weight_count": (C.c_int, [U32, U32, U32, PU64]),
            "bvs_mlp_init": (C.c_int, [U32, U32, U32, U64, P, P]),
            "bvs_learned_index_bytes": (C.c_int, [P, U32, U64, U64, PU64]),
            "bvs_learned_build_workspace_bytes": (C.c_int, [P, U32, U64, U64, PU64]),
            "bvs_build_index_learned": (C.c_int, [P, U32, P, P, P, U64, P, U64, P, U64, P, C.POINTER(P)]),
            "bvs_train_workspace_bytes": (C.c_int, [P, U64, PU64]),
            "bvs_train_gradients": (C.c_int, [P, P, P, U64, P, U32, P, P, C.POINTER(C.c_float), P, U64, P]),
            "bvs_train_projection": (C.c_int, [P, P, P, U64, P, U64, P, P, U64, P, P]),
            "bvs_train_state_bytes": (C.c_int, [P, PU64]),
            "bvs_train_state_init": (C.c_int, [P, P, P]),
            "bvs_train_projection_resume": (C.c_int, [P, P, P, U64, P, U64, P, P, P, U64, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != BVS_OK:
        raise BvsError(status, lib().bvs_last_error().decode())


def _ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _offsets(off) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(off, dtype=np.uint64))
    return a


def _u64p(a: np.ndarray):
    return a.ctypes.data_as(PU64)


def projection(params: Params) -> np.ndarray:
    L, s = params.code_bits, params.fan_in
    out = np.zeros((L, s), np.uint16)
    check(lib().bvs_projection(C.byref(params), out.ctypes.data_as(C.c_void_p)))
    return out


PROFILE_TIMING, PROFILE_COUNTERS = 1, 2


def profile_enable(on: bool = True, counters: bool = False) -> None:
    """Reset the table and start (or stop) per-stage HIP-event timing and,
    separately, the work counters."""
    check(lib().bvs_profile_enable((PROFILE_TIMING if on else 0) | (PROFILE_COUNTERS if counters else 0)))


def profile_read() -> dict:
    """{stage name: (total ms, calls)} accumulated since profile_enable."""
    t = StageTimes()
    check(lib().bvs_profile_read(C.byref(t)))
    return {lib().bvs_stage_name(i).decode(): (float(t.ms[i]), int(t.calls[i])) for i in range(N_STAGES)}


def profile_counters() -> dict:
    """Work counters accumulated since profile_enable."""
    t = StageTimes()
    check(lib().bvs_profile_read(C.byref(t)))
    return {COUNTER_NAMES[i]: int(t.counters[i]) for i in range(N_COUNTERS)}


def params_check(params: Params) -> None:
    check(lib().bvs_params_check(C.byref(params)))


def _bytes(fn, *args) -> int:
    out = C.c_uint64(0)
    check(fn(*args, C.byref(out)))
    return int(out.value)


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


class Index:
    """A built index.  `vectors` is a float32 CUDA tensor [N, dim] on the
    2^-12 grid; `offsets` host offsets [n + 1]."""

    def __init__(self, params: Params, vectors: torch.Tensor, offsets, stream=None, mlp=None):
        """mlp: optional (hidden, float32 packed weights tensor) of a learned projection."""
        L = lib()
        if not (vectors.is_cuda and vectors.dtype == torch.float32 and vectors.is_contiguous()):
            raise ValueError("vectors must be a contiguous float32 CUDA tensor")
        self.params = Params.from_buffer_copy(params)
        self.device = vectors.device
        off = _offsets(offsets)
        n = len(off) - 1
        N = int(off[-1]) if n >= 0 else 0
        h = C.c_void_p()
        if mlp is None:
            nbytes = _bytes(L.bvs_index_bytes, C.byref(self.params), n, N)
            wbytes = _bytes(L.bvs_build_workspace_bytes, C.byref(self.params), n, N)
            self.mem = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            ws = _workspace(wbytes, self.device)
            check(L.bvs_build_index(C.byref(self.params), _ptr(vectors), _u64p(off), n, _ptr(self.mem), nbytes,
                                    _ptr(ws), ws.numel(), _stream(stream), C.byref(h)))
        else:
            hidden, weights = mlp
            nbytes = _bytes(L.bvs_learned_index_bytes, C.byref(self.params), hidden, n, N)
            wbytes = _bytes(L.bvs_learned_build_workspace_bytes, C.byref(self.params), hidden, n, N)
            self.mem = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            ws = _workspace(wbytes, self.device)
            check(L.bvs_build_index_learned(C.byref(self.params), hidden, _ptr(weights), _ptr(vectors), _u64p(off),
                                            n, _ptr(self.mem), nbytes, _ptr(ws), ws.numel(), _stream(stream),
                                            C.byref(h)))
        self._h = h
        del ws
        info = IndexInfo()
        check(L.bvs_index_get_info(self._h, C.byref(info)))
        self.n_sets, self.n_vectors, self.ld = int(info.n_sets), int(info.n_vectors), int(info.ld_sets)
        self.dim_padded, self.max_set_size = int(info.dim_padded), int(info.max_set_size)

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None):
            lib().bvs_index_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- inspection
    def sketch_views(self):
        """(count uint8 [L, ld], bits int64 [L/128, ld, 2]) views into the index memory."""
        c, b = C.c_void_p(), C.c_void_p()
        check(lib().bvs_sketch_views(self._h, C.byref(c), C.byref(b)))
        base = self.mem.data_ptr()
        Lb = self.params.code_bits
        cnt = self.mem[c.value - base: c.value - base + Lb * self.ld].view(Lb, self.ld)
        nb = (Lb // 64) * self.ld * 8
        bits = self.mem[b.value - base: b.value - base + nb].view(torch.int64).view(Lb // 128, self.ld, 2)
        return cnt, bits

    def encode(self, x: torch.Tensor, stream=None) -> torch.Tensor:
        """Codes int64 [n, L/64] (bit j % 64 of word j / 64 is output j)."""
        n = x.shape[0]
        out = torch.empty(n, self.params.code_bits // 64, dtype=torch.int64, device=self.device)
        wb = _bytes(lib().bvs_encode_workspace_bytes, self._h, n)
        ws = _workspace(wb, self.device)
        check(lib().bvs_encode(self._h, _ptr(x), n, _ptr(ws), ws.numel(), _ptr(out), _stream(stream)))
        return out

    def _qargs(self, q: torch.Tensor, q_offsets):
        if not (q.is_cuda and q.dtype == torch.float32 and q.is_contiguous()):
            raise ValueError("queries must be a contiguous float32 CUDA tensor")
        off = _offsets(q_offsets)
        return off, len(off) - 1, int(off[-1])

    def search_workspace(self, n_q: int, n_q_vectors: int) -> torch.Tensor:
        return _workspace(_bytes(lib().bvs_search_workspace_bytes, self._h, n_q, n_q_vectors), self.device)

    def brute_workspace(self, n_q: int, n_q_vectors: int) -> torch.Tensor:
        return _workspace(_bytes(lib().bvs_bruteforce_workspace_bytes, self._h, n_q, n_q_vectors), self.device)

    def query_sketch(self, q, q_offsets, stream=None):
        off, n_q, NQ = self._qargs(q, q_offsets)
        L, A = self.params.code_bits, self.params.access_lists
        cq = torch.empty(n_q, L, dtype=torch.int16, device=self.device)
        sq = torch.empty(n_q, L // 64, dtype=torch.int64, device=self.device)
        pos = torch.empty(n_q, A, dtype=torch.int32, device=self.device)
        ws = self.search_workspace(n_q, NQ)
        check(lib().bvs_query_sketch(self._h, _ptr(q), _u64p(off), n_q, _ptr(ws), ws.numel(), _ptr(cq),
                                     _ptr(sq), _ptr(pos), _stream(stream)))
        return cq, sq, pos

    def candidates(self, q, q_offsets, stream=None):
        """F2 per query: ids int32 [n_q, T], scores int16 [n_q, T], count int32 [n_q]."""
        off, n_q, NQ = self._qargs(q, q_offsets)
        T = self.params.top_t
        ids = torch.empty(n_q, T, dtype=torch.int32, device=self.device)
        sc = torch.empty(n_q, T, dtype=torch.int16, device=self.device)
        cnt = torch.empty(n_q, dtype=torch.int32, device=self.device)
        ws = self.search_workspace(n_q, NQ)
        check(lib().bvs_search_candidates(self._h, _ptr(q), _u64p(off), n_q, _ptr(ws), ws.numel(), _ptr(ids),
                                          _ptr(sc), _ptr(cnt), _stream(stream)))
        return ids, sc, cnt

    def search(self, q, q_offsets, k: int, ws: torch.Tensor | None = None, out=None, stream=None):
        """Top-k per query: ids int32 [n_q, k], dist float32 [n_q, k], count int32 [n_q]."""
        off, n_q, NQ = self._qargs(q, q_offsets)
        if ws is None:
            ws = self.search_workspace(n_q, NQ)
        if out is None:
            out = (torch.empty(n_q, k, dtype=torch.int32, device=self.device),
                   torch.empty(n_q, k, dtype=torch.float32, device=self.device),
                   torch.empty(n_q, dtype=torch.int32, device=self.device))
        ids, dist, cnt = out
        check(lib().bvs_search(self._h, _ptr(q), _u64p(off), n_q, k, _ptr(ws), ws.numel(), _ptr(ids),
                               _ptr(dist), _ptr(cnt), _stream(stream)))
        return ids, dist, cnt

    def search_noalloc(self, q, q_offsets, k: int, out=None, stream=None):
        """bvs_search_noalloc: the search of `search` on the library's fixed
        device scratch (no workspace argument; outputs as for `search`)."""
        off, n_q, NQ = self._qargs(q, q_offsets)
        if out is None:
            out = (torch.empty(n_q, k, dtype=torch.int32, device=self.device),
                   torch.empty(n_q, k, dtype=torch.float32, device=self.device),
                   torch.empty(n_q, dtype=torch.int32, device=self.device))
        ids, dist, cnt = out
        check(lib().bvs_search_noalloc(self._h, _ptr(q), _u64p(off), n_q, k, _ptr(ids), _ptr(dist), _ptr(cnt),
                                       _stream(stream)))
        return ids, dist, cnt

    def set_search_params(self, access_lists: int, min_count: int, top_t: int):
        """A, M and T of later searches (no rebuild; workspaces must be sized again)."""
        check(lib().bvs_index_set_search_params(self._h, access_lists, min_count, top_t))
        self.params.access_lists, self.params.min_count, self.params.top_t = access_lists, min_count, top_t

    # -- inverted lists (Def. 9, Alg. 4)
    def attach_lists(self, stream=None) -> int:
        """Build the inverted lists of the count Bloom filters into new device memory."""
        wb = _bytes(lib().bvs_lists_workspace_bytes, self._h)
        ws = _workspace(wb, self.device)
        out = C.c_uint64(0)
        check(lib().bvs_lists_bytes(self._h, _ptr(ws), ws.numel(), _stream(stream), C.byref(out)))
        nbytes = int(out.value)
        mem = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        check(lib().bvs_lists_attach(self._h, _ptr(mem), nbytes, _ptr(ws), ws.numel(), _stream(stream)))
        self._lists = mem
        return nbytes

    def lists_views(self):
        """(cum int32 [L, 257], start int64 [L + 1], ids int32 [nnz]) views of the attached lists."""
        a, b, c, n = C.c_void_p(), C.c_void_p(), C.c_void_p(), C.c_uint64(0)
        check(lib().bvs_lists_views(self._h, C.byref(a), C.byref(b), C.byref(c), C.byref(n)))
        base = self._lists.data_ptr()
        L = self.params.code_bits
        nnz = int(n.value)

        def view(ptr, count, dtype, size):
            off = ptr - base
            return self._lists[off: off + count * size].view(dtype)
        return (view(a.value, L * 257, torch.int32, 4).view(L, 257), view(b.value, L + 1, torch.int64, 8),
                view(c.value, nnz, torch.int32, 4))

    def set_first_layer(self, mode: str):
        """"bitmaps" (default) or "lists" (needs attach_lists)."""
        check(lib().bvs_index_set_first_layer(self._h, FIRST_LAYER[mode]))

    # -- full scan (Alg. 2)
    def attach_codes(self, stream=None) -> int:
        """Encode every database vector into sparse codes for the full scan."""
        nbytes = _bytes(lib().bvs_codes_bytes, self._h)
        wbytes = _bytes(lib().bvs_codes_attach_workspace_bytes, self._h)
        mem = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        ws = _workspace(wbytes, self.device)
        check(lib().bvs_codes_attach(self._h, _ptr(mem), nbytes, _ptr(ws), ws.numel(), _stream(stream)))
        self._codes = mem
        return nbytes

    def full_workspace(self, n_q: int, n_q_vectors: int) -> torch.Tensor:
        return _workspace(_bytes(lib().bvs_search_full_workspace_bytes, self._h, n_q, n_q_vectors), self.device)

    def full_scores(self, q, q_offsets, stream=None) -> torch.Tensor:
        """Haus^H of every query to every set, int16 [n_q, n_sets] (uint16 values)."""
        off, n_q, NQ = self._qargs(q, q_offsets)
        out = torch.empty(n_q, self.n_sets, dtype=torch.int16, device=self.device)
        ws = self.full_workspace(n_q, NQ)
        check(lib().bvs_full_scores(self._h, _ptr(q), _u64p(off), n_q, _ptr(ws), ws.numel(), _ptr(out),
                                    _stream(stream)))
        return out

    def full_candidates(self, q, q_offsets, stream=None):
        """F of Alg. 2 per query: ids int32 [n_q, T], scores int16 [n_q, T], count int32 [n_q]."""
        off, n_q, NQ = self._qargs(q, q_offsets)
        T = self.params.top_t
        ids = torch.empty(n_q, T, dtype=torch.int32, device=self.device)
        sc = torch.empty(n_q, T, dtype=torch.int16, device=self.device)
        cnt = torch.empty(n_q, dtype=torch.int32, device=self.device)
        ws = self.full_workspace(n_q, NQ)
        check(lib().bvs_search_full_candidates(self._h, _ptr(q), _u64p(off), n_q, _ptr(ws), ws.numel(), _ptr(ids),
                                               _ptr(sc), _ptr(cnt), _stream(stream)))
        return ids, sc, cnt

    def search_full(self, q, q_offsets, k: int, ws: torch.Tensor | None = None, out=None, stream=None):
        """Alg. 2 top-k per query; outputs as for `search`."""
        off, n_q, NQ = self._qargs(q, q_offsets)
        ws = self.full_workspace(n_q, NQ) if ws is None else ws
        ids, dist, cnt = self._outs(n_q, k) if out is None else out
        check(lib().bvs_search_full(self._h, _ptr(q), _u64p(off), n_q, k, _ptr(ws), ws.numel(), _ptr(ids),
                                    _ptr(dist), _ptr(cnt), _stream(stream)))
        return ids, dist, cnt

    # -- precision form
    def attach_lowp(self, fmt: str, stream=None):
        """Build and attach the BF16 ("bf16") or FP8 E4M3 ("fp8") copy of the vectors."""
        f = LOWP[fmt]
        nbytes = _bytes(lib().bvs_lowp_bytes, self._h, f)
        mem = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        check(lib().bvs_lowp_attach(self._h, f, _ptr(mem), nbytes, _stream(stream)))
        self.__dict__.setdefault("_lowp", {})[fmt] = mem
        return nbytes

    def lowp_workspace(self, n_q: int, n_q_vectors: int) -> torch.Tensor:
        return _workspace(_bytes(lib().bvs_lowp_workspace_bytes, self._h, n_q, n_q_vectors), self.device)

    def search_lowp(self, q, q_offsets, k: int, fmt: str, margin: float = 0.02, ws: torch.Tensor | None = None,
                    out=None, stream=None):
        """(ids, dist, count, rechecked) of the precision form."""
        off, n_q, NQ = self._qargs(q, q_offsets)
        if ws is None:
            ws = self.lowp_workspace(n_q, NQ)
        if out is None:
            out = (torch.empty(n_q, k, dtype=torch.int32, device=self.device),
                   torch.empty(n_q, k, dtype=torch.float32, device=self.device),
                   torch.empty(n_q, dtype=torch.int32, device=self.device),
                   torch.empty(n_q, dtype=torch.int32, device=self.device))
        ids, dist, cnt, rech = out
        check(lib().bvs_search_lowp(self._h, LOWP[fmt], margin, _ptr(q), _u64p(off), n_q, k, _ptr(ws), ws.numel(),
                                    _ptr(ids), _ptr(dist), _ptr(cnt), _ptr(rech), _stream(stream)))
        return ids, dist, cnt, rech

    def hausdorff_lowp(self, q, q_offsets, ids: torch.Tensor, fmt: str, stream=None) -> torch.Tensor:
        """Approximate squared Hausdorff values float32 [n_q, m] against ids int32 [n_q, m]."""
        off, n_q, NQ = self._qargs(q, q_offsets)
        ids = ids.to(torch.int32).contiguous()
        m = ids.shape[1]
        out = torch.empty(n_q, m, dtype=torch.float32, device=self.device)
        ws = self.lowp_workspace(n_q, NQ)
        check(lib().bvs_hausdorff_lowp(self._h, LOWP[fmt], _ptr(q), _u64p(off), n_q, _ptr(ids), m, _ptr(ws),
                                       ws.numel(), _ptr(out), _stream(stream)))
        return out

    def bruteforce(self, q, q_offsets, k: int, ws: torch.Tensor | None = None, out=None, stream=None):
        off, n_q, NQ = self._qargs(q, q_offsets)
        if ws is None:
            ws = self.brute_workspace(n_q, NQ)
        if out is None:
            out = (torch.empty(n_q, k, dtype=torch.int32, device=self.device),
                   torch.empty(n_q, k, dtype=torch.float32, device=self.device),
                   torch.empty(n_q, dtype=torch.int32, device=self.device))
        ids, dist, cnt = out
        check(lib().bvs_bruteforce(self._h, _ptr(q), _u64p(off), n_q, k, _ptr(ws), ws.numel(), _ptr(ids),
                                   _ptr(dist), _ptr(cnt), _stream(stream)))
        return ids, dist, cnt

    def _outs(self, n_q, k):
        return (torch.empty(n_q, k, dtype=torch.int32, device=self.device),
                torch.empty(n_q, k, dtype=torch.float32, device=self.device),
                torch.empty(n_q, dtype=torch.int32, device=self.device))

    def search_metric(self, q, q_offsets, k: int, metric: str, ws: torch.Tensor | None = None, out=None,
                      stream=None):
        """Cascade search re-ranked by `metric` ("hausdorff", "meanmin", "min")."""
        off, n_q, NQ = self._qargs(q, q_offsets)
        ws = self.search_workspace(n_q, NQ) if ws is None else ws
        ids, dist, cnt = self._outs(n_q, k) if out is None else out
        check(lib().bvs_search_metric(self._h, METRIC[metric], _ptr(q), _u64p(off), n_q, k, _ptr(ws), ws.numel(),
                                      _ptr(ids), _ptr(dist), _ptr(cnt), _stream(stream)))
        return ids, dist, cnt

    def bruteforce_metric(self, q, q_offsets, k: int, metric: str, ws: torch.Tensor | None = None, out=None,
                          stream=None):
        """Exact top-k over every set by `metric`."""
        off, n_q, NQ = self._qargs(q, q_offsets)
        ws = self.brute_workspace(n_q, NQ) if ws is None else ws
        ids, dist, cnt = self._outs(n_q, k) if out is None else out
        check(lib().bvs_bruteforce_metric(self._h, METRIC[metric], _ptr(q), _u64p(off), n_q, k, _ptr(ws),
                                          ws.numel(), _ptr(ids), _ptr(dist), _ptr(cnt), _stream(stream)))
        return ids, dist, cnt

    def hausdorff_all(self, q, q_offsets, stream=None) -> torch.Tensor:
        """2^24 * Hausdorff^2 of every (query, set) pair, int32 [n_q, n_sets] (values < 2^28)."""
        off, n_q, NQ = self._qargs(q, q_offsets)
        out = torch.empty(n_q, self.n_sets, dtype=torch.int32, device=self.device)
        ws = self.brute_workspace(n_q, NQ)
        check(lib().bvs_hausdorff_all(self._h, _ptr(q), _u64p(off), n_q, _ptr(ws), ws.numel(), _ptr(out),
                                      _stream(stream)))
        return out


def as_u64(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def as_u32(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def as_u16(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint16)


class Batch:
    """A batched search plan over one index (bvs_batch_*): the whole cascade
    for many query sets, the re-rank as one persistent launch or as the phase
    sequence of Index.search by size class (phases=True, or the autotuner's
    choice), optionally captured once in a hipGraph.  Outputs as for
    Index.search.  Graph capture needs a non-default stream; by default the
    plan makes its own."""

    def __init__(self, index: Index, q: torch.Tensor, q_offsets, k: int, lds_rows: int = 0, waves: int = 0,
                 graph: bool = True, stream=None, phases: bool = False):
        L = lib()
        self.index = index
        off, n_q, NQ = index._qargs(q, q_offsets)
        self.n_q, self.k = n_q, k
        self.q = q
        cfg = BatchConfig(lds_rows, waves, 1 if graph else 0, BVS_BATCH_PHASES if phases else 0)
        h = C.c_void_p()
        check(L.bvs_batch_create(index._h, _u64p(off), n_q, k, C.byref(cfg), C.byref(h)))
        self._h = h
        if stream is None and graph:
            stream = torch.cuda.Stream(device=index.device)
        self.stream = stream
        info = self.info()
        self.ws = _workspace(int(info["workspace_bytes"]), index.device)
        dev = index.device
        self.ids = torch.empty(n_q, k, dtype=torch.int32, device=dev)
        self.dist = torch.empty(n_q, k, dtype=torch.float32, device=dev)
        self.count = torch.empty(n_q, dtype=torch.int32, device=dev)
        st = self._stream_obj()
        st.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(st):
            check(L.bvs_batch_bind(self._h, _ptr(q), _ptr(self.ws), self.ws.numel(), _ptr(self.ids),
                                   _ptr(self.dist), _ptr(self.count), _stream(st)))

    def _stream_obj(self):
        return self.stream if self.stream is not None else torch.cuda.current_stream(self.index.device)

    def launch(self):
        """Enqueue one batched search (no synchronisation)."""
        st = self._stream_obj()
        st.wait_stream(torch.cuda.current_stream(self.index.device))
        check(lib().bvs_batch_launch(self._h, _stream(st)))
        torch.cuda.current_stream(self.index.device).wait_stream(st)

    def status(self):
        """Synchronise and raise BvsError on bad query data."""
        check(lib().bvs_batch_status(self._h, _stream(self._stream_obj())))

    def run(self):
        """One launch, synchronised; returns (ids, dist, count)."""
        self.launch()
        self.status()
        return self.ids, self.dist, self.count

    def info(self) -> dict:
        i = BatchInfo()
        check(lib().bvs_batch_get_info(self._h, C.byref(i)))
        n = int(i.n_tried)
        return dict(n_q=int(i.n_q), max_rows=int(i.max_rows), n_q_vectors=int(i.n_q_vectors),
                    workspace_bytes=int(i.workspace_bytes), lds_rows=int(i.lds_rows), waves=int(i.waves),
                    blocks=int(i.blocks), from_cache=bool(i.from_cache), graph=bool(i.graph),
                    tried=[(int(i.tried_lds_rows[j]), int(i.tried_waves[j]), float(i.tried_ms[j]))
                           for j in range(n)])

    def close(self):
        if getattr(self, "_h", None):
            lib().bvs_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# -- learned projection
def mlp_weights(dim: int, hidden: int, code_bits: int, seed: int = 0, device="cuda") -> torch.Tensor:
    """Initialised packed float32 weights [W1 | b1 | W2 | b2]."""
    n = C.c_uint64()
    check(lib().bvs_mlp_weight_count(dim, hidden, code_bits, C.byref(n)))
    w = torch.empty(int(n.value), dtype=torch.float32, device=device)
    check(lib().bvs_mlp_init(dim, hidden, code_bits, seed, _ptr(w), _stream(None)))
    return w


def unpack_mlp(w: torch.Tensor, dim: int, hidden: int, code_bits: int):
    a = hidden * dim
    b = a + hidden
    c = b + code_bits * hidden
    return (w[:a].view(hidden, dim), w[a:b], w[b:c].view(code_bits, hidden), w[c:])


class Trainer:
    """Triplet training of the learned projection on a training collection
    (float32 CUDA vectors, host offsets); triplets uint32 [n, 3] of set ids."""

    def __init__(self, cfg: TrainConfig, vectors: torch.Tensor, offsets, max_batch_rows: int):
        self.cfg = TrainConfig.from_buffer_copy(cfg)
        self.vectors = vectors
        self.off = _offsets(offsets)
        nb = C.c_uint64()
        check(lib().bvs_train_workspace_bytes(C.byref(self.cfg), max_batch_rows, C.byref(nb)))
        self.ws = _workspace(int(nb.value), vectors.device)

    def gradients(self, weights: torch.Tensor, triplets: np.ndarray):
        trip = np.ascontiguousarray(np.asarray(triplets, np.uint32))
        grads = torch.empty_like(weights)
        loss = C.c_float()
        check(lib().bvs_train_gradients(C.byref(self.cfg), _ptr(self.vectors), _u64p(self.off), len(self.off) - 1,
                                        trip.ctypes.data_as(C.c_void_p), len(trip), _ptr(weights), _ptr(grads),
                                        C.byref(loss), _ptr(self.ws), self.ws.numel(), _stream(None)))
        return float(loss.value), grads

    def new_state(self) -> torch.Tensor:
        """A zeroed training state (Adam moments, step and epoch counts)."""
        st = torch.empty(_bytes(lib().bvs_train_state_bytes, C.byref(self.cfg)), dtype=torch.uint8,
                         device=self.vectors.device)
        check(lib().bvs_train_state_init(C.byref(self.cfg), _ptr(st), _stream(None)))
        return st

    def train_resume(self, weights: torch.Tensor, triplets: np.ndarray, state: torch.Tensor):
        """cfg.epochs more epochs from `state` (updated in place)."""
        trip = np.ascontiguousarray(np.asarray(triplets, np.uint32))
        losses = (C.c_float * max(1, self.cfg.epochs))()
        check(lib().bvs_train_projection_resume(C.byref(self.cfg), _ptr(self.vectors), _u64p(self.off),
                                                len(self.off) - 1, trip.ctypes.data_as(C.c_void_p), len(trip),
                                                _ptr(weights), _ptr(state), _ptr(self.ws), self.ws.numel(), losses,
                                                _stream(None)))
        return [float(x) for x in losses[: self.cfg.epochs]]

    def train(self, weights: torch.Tensor, triplets: np.ndarray):
        trip = np.ascontiguousarray(np.asarray(triplets, np.uint32))
        losses = (C.c_float * max(1, self.cfg.epochs))()
        check(lib().bvs_train_projection(C.byref(self.cfg), _ptr(self.vectors), _u64p(self.off), len(self.off) - 1,
                                         trip.ctypes.data_as(C.c_void_p), len(trip), _ptr(weights), _ptr(self.ws),
                                         self.ws.numel(), losses, _stream(None)))
        return [float(x) for x in losses[: self.cfg.epochs]]
