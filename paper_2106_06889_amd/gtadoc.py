"""Python binding of libgtadoc (ctypes). Argument marshalling only: every
step of every query runs in the library's HIP kernels. torch provides the
device memory (the arena and the output tensors) and the streams.

Loading fails loudly when the HIP library has not been built; there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
import sys
import weakref
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgtadoc.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "gtadoc.h")

OK = 0
ERR_INVALID_ARG, ERR_BAD_GRAMMAR, ERR_CYCLE, ERR_OOM, ERR_UNSUPPORTED, ERR_OVERFLOW, ERR_HIP = range(-1, -8, -1)
IN_HOST, IN_DEVICE, IN_BORROW, LOAD_LEVELS = 0x1, 0x2, 0x4, 0x8
_NAMES = {-1: "INVALID_ARG", -2: "BAD_GRAMMAR", -3: "CYCLE", -4: "OOM", -5: "UNSUPPORTED", -6: "OVERFLOW", -7: "HIP"}


class GtadocError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"gtadoc error {_NAMES.get(code, code)}: {message}")
        self.code = code


class Stats(ctypes.Structure):
    _fields_ = [("tokens", ctypes.c_int64), ("symbols", ctypes.c_int64), ("rules", ctypes.c_int64),
                ("files", ctypes.c_int64), ("word_syms", ctypes.c_int64), ("root_syms", ctypes.c_int64),
                ("depth", ctypes.c_int64), ("vocab", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("arena_bytes", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


_lib = None
_vp, _i64, _i32, _u32, _u64, _int = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32,
                                     ctypes.c_uint64, ctypes.c_int)

EXPORTS = {
    "gtadoc_ctx_create": [_vp, _u64, _vp],
    "gtadoc_ctx_destroy": [_vp],
    "gtadoc_ctx_usage": [_vp, _vp, _vp, _vp],
    "gtadoc_load_grammar": [_vp, _vp, _i64, _vp, _i64, _vp, _i64, _i32, _u32, _vp, _vp],
    "gtadoc_grammar_stats": [_vp, _vp],
    "gtadoc_build_levels": [_vp, _vp],
    "gtadoc_grammar_edges": [_vp, _vp, _vp],
    "gtadoc_query_bytes": [_vp, _int, _int, _int, _vp, _vp],
    "gtadoc_free_grammar": [_vp],
    "gtadoc_word_count": [_vp, _vp, _vp],
    "gtadoc_word_count_noalloc": [_vp, _vp, _vp],
    "gtadoc_decompress": [_vp, _vp, _vp, _vp],
    "gtadoc_sort": [_vp, _vp, _vp, _vp, _vp, _vp],
    "gtadoc_term_vector": [_vp, _vp, _vp],
    "gtadoc_term_vector_ex": [_vp, _int, _vp, _vp],
    "gtadoc_term_vector_strategy": [_vp, _vp],
    "gtadoc_inverted_index": [_vp, _vp, _vp],
    "gtadoc_inverted_index_from_tv": [_vp, _vp, _vp, _vp],
    "gtadoc_ranked_inverted_index": [_vp, _vp, _vp],
    "gtadoc_ranked_inverted_index_from_tv": [_vp, _vp, _vp, _vp],
    "gtadoc_sequence_count": [_vp, _int, _vp, _vp],
    "gtadoc_sequence_count_wide": [_vp, _int, _vp, _vp],
    "gtadoc_result_array": [_vp, _int, _vp, _vp, _vp],
    "gtadoc_result_free": [_vp],
    "gtadoc_ctx_set_param": [_vp, _int, _i64],
    "gtadoc_ctx_get_param": [_vp, _int, _vp],
    "gtadoc_batch_create": [_vp, _int, _u64, _vp],
    "gtadoc_batch_word_count": [_vp, _vp, _vp, _int, _vp],
    "gtadoc_batch_destroy": [_vp],
    "gtadoc_batch_submit": [_vp, _vp, _int, _vp],
    "gtadoc_ctx_phase_time": [_vp, _int, _vp, _vp, _int],
    "gtadoc_last_error": [],
}
PARAM_WC_CHUNK, PARAM_BATCH_BLOCKS_PER_CU, PARAM_BATCH_GRAPH, PARAM_TIMING, PARAM_LEVEL_WIDE = 1, 2, 3, 4, 5
PARAM_LEVEL_LONG_BODY, PARAM_LEVEL_MID_RULES, PARAM_LEVEL_MID_BLOCKS, PARAM_LEVEL_TAIL_RULES = 6, 7, 8, 9
PARAM_FLOW_KEEP, PARAM_FLOW_GROUP, PARAM_FLOW_CHUNK = 10, 11, 12
PHASES = {"levels": 0, "word_count": 1, "sort": 2, "seq_windows": 3, "tv_tables": 4, "tv_reduce": 5, "load": 6,
          "decompress": 7, "tv_topdown": 8}


def timing_mask(*phases: str) -> int:
    """PARAM_TIMING value that times only the named phases (bit p + 1 per phase p)."""
    return sum(2 << PHASES[p] for p in set(phases))


TV_AUTO, TV_BOTTOM_UP, TV_TOP_DOWN = 0, 1, 2
(QUERY_WORD_COUNT, QUERY_TERM_VECTOR, QUERY_SEQUENCE_COUNT, QUERY_INVERTED_INDEX,
 QUERY_RANKED_INVERTED_INDEX) = 1, 2, 3, 4, 5


class QueryStruct(ctypes.Structure):
    """gtadoc_query of the C ABI."""
    _fields_ = [("grammar", ctypes.c_void_p), ("kind", ctypes.c_int32), ("n", ctypes.c_int32),
                ("counts", ctypes.c_void_p), ("result", ctypes.c_void_p), ("status", ctypes.c_int32),
                ("strategy", ctypes.c_int32)]


def lib() -> ctypes.CDLL:
    """The loaded HIP library. Raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m paper_2106_06889_amd.build)")
        l = ctypes.CDLL(LIB_PATH)
        for name, args in EXPORTS.items():
            fn = getattr(l, name)
            fn.argtypes = args
            fn.restype = ctypes.c_char_p if name == "gtadoc_last_error" else ctypes.c_int
        _lib = l
    return _lib


def _check(rc: int):
    if rc != OK:
        raise GtadocError(rc, lib().gtadoc_last_error().decode())


def _stream_ptr(stream) -> int | None:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dev_tensor(ptr: int, n: int, elem_bytes: int, owner: torch.Tensor) -> torch.Tensor:
    """A view of n elements at device address ptr inside `owner` (the arena)."""
    off = ptr - owner.data_ptr()
    dtype = {4: torch.int32, 8: torch.int64}[elem_bytes]
    if n == 0:
        return torch.empty(0, dtype=dtype, device=owner.device)
    return owner[off:off + n * elem_bytes].view(dtype)


class Context:
    """A gtadoc context over a torch-owned device arena."""

    def __init__(self, arena_bytes: int, device: int | str | torch.device = "cuda"):
        self.device = torch.device(device) if not isinstance(device, int) else torch.device("cuda", device)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        h = _vp()
        with torch.cuda.device(self.device):
            _check(lib().gtadoc_ctx_create(self.arena.data_ptr(), int(arena_bytes), ctypes.byref(h)))
        self.handle = h
        self._children = weakref.WeakSet()  # grammars, results and plans living in the arena

    def close(self):
        """Release every grammar, result and batch plan still open on the
        context, then the context (they must not outlive it)."""
        if self.handle:
            for c in list(self._children):
                c.free()
            lib().gtadoc_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        # no HIP call during interpreter shutdown: the runtime (and a
        # profiler's tool library) may already be torn down
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def set_param(self, param: int, value: int):
        _check(lib().gtadoc_ctx_set_param(self.handle, int(param), int(value)))

    def get_param(self, param: int) -> int:
        v = _i64()
        _check(lib().gtadoc_ctx_get_param(self.handle, int(param), ctypes.byref(v)))
        return v.value

    def phase_time(self, phase: str, reset: bool = False) -> tuple[float, int]:
        """(summed device ms, occurrences) of a timed phase; needs PARAM_TIMING on."""
        ms, n = ctypes.c_double(), _i64()
        _check(lib().gtadoc_ctx_phase_time(self.handle, PHASES[phase], ctypes.byref(ms), ctypes.byref(n), int(reset)))
        return ms.value, n.value

    def batch(self, max_items: int, max_entries: int) -> "Batch":
        return Batch(self, max_items, max_entries)

    def usage(self) -> tuple[int, int, int]:
        a, b, c = _u64(), _u64(), _u64()
        _check(lib().gtadoc_ctx_usage(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def load(self, rule_off, sym, file_off, vocab: int, stream=None, borrow: bool = False,
             levels: bool = False) -> "Grammar":
        """Load a grammar from numpy arrays (host) or torch device tensors.
        levels=True builds the level structure during the load (level walk);
        otherwise the weights come from the dataflow walk and the levels are
        built when a query first needs them."""
        keep = ()
        if isinstance(sym, torch.Tensor):
            rule_off = rule_off.to(torch.int64).contiguous()
            sym = sym.to(torch.int32).contiguous()
            file_off = file_off.to(torch.int64).contiguous()
            flags = IN_DEVICE | (IN_BORROW if borrow else 0)
            ptrs = (rule_off.data_ptr(), sym.data_ptr() if sym.numel() else None, file_off.data_ptr())
            keep = (rule_off, sym, file_off) if borrow else ()
        else:
            rule_off = np.ascontiguousarray(rule_off, dtype=np.int64)
            sym = np.ascontiguousarray(sym, dtype=np.int32)
            file_off = np.ascontiguousarray(file_off, dtype=np.int64)
            flags = IN_HOST
            ptrs = (rule_off.ctypes.data, sym.ctypes.data if sym.size else None, file_off.ctypes.data)
        if levels:
            flags |= LOAD_LEVELS
        R, S, F = len(rule_off) - 1, len(sym), len(file_off) - 1
        h = _vp()
        with torch.cuda.device(self.device):
            _check(lib().gtadoc_load_grammar(self.handle, ptrs[0], R, ptrs[1], S, ptrs[2], F, int(vocab), flags,
                                             _stream_ptr(stream), ctypes.byref(h)))
        return Grammar(self, h, keep)


@dataclass(eq=False)
class Result:
    arrays: list
    handle: object
    ctx: Context

    def __post_init__(self):
        self.ctx._children.add(self)

    def length(self, index: int) -> int:
        return int(self.arrays[index].numel())

    def free(self):
        if self.handle and self.ctx.handle:
            lib().gtadoc_result_free(self.handle)
        self.handle = None


class Grammar:
    def __init__(self, ctx: Context, handle, keep=()):
        self.ctx, self.handle, self._keep = ctx, handle, keep
        ctx._children.add(self)
        st = Stats()
        _check(lib().gtadoc_grammar_stats(handle, ctypes.byref(st)))
        self.stats = st.as_dict()
        self.vocab = st.vocab

    def free(self):
        if self.handle and self.ctx.handle:
            lib().gtadoc_free_grammar(self.handle)
        self.handle = None

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.free()
        except Exception:
            pass

    def build_levels(self, stream=None) -> int:
        """Builds the level structure if the load did not; returns the depth
        (also refreshed in self.stats)."""
        _check(lib().gtadoc_build_levels(self.handle, _stream_ptr(stream)))
        st = Stats()
        _check(lib().gtadoc_grammar_stats(self.handle, ctypes.byref(st)))
        self.stats = st.as_dict()
        return int(self.stats["depth"])

    def word_count(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """uint64 counts as an int64 tensor of vocab entries (bit pattern = uint64)."""
        if out is None:
            out = torch.empty(self.vocab, dtype=torch.int64, device=self.ctx.device)
        assert out.dtype == torch.int64 and out.numel() == self.vocab and out.is_contiguous()
        _check(lib().gtadoc_word_count(self.handle, out.data_ptr(), _stream_ptr(stream)))
        return out

    def word_count_noalloc(self, out: torch.Tensor, stream=None) -> torch.Tensor:
        """Word count into the caller's int64 tensor of vocab entries, with the
        library's static device scratch instead of arena memory."""
        assert out.dtype == torch.int64 and out.numel() == self.vocab and out.is_contiguous()
        _check(lib().gtadoc_word_count_noalloc(self.handle, out.data_ptr(), _stream_ptr(stream)))
        return out

    def decompress(self, stream=None) -> tuple[torch.Tensor, torch.Tensor]:
        """The text the grammar spells, on the device: (tokens int32[T],
        file_off int64[F+1])."""
        T, F = int(self.stats["tokens"]), int(self.stats["files"])
        tokens = torch.empty(max(T, 1), dtype=torch.int32, device=self.ctx.device)
        file_off = torch.empty(F + 1, dtype=torch.int64, device=self.ctx.device)
        _check(lib().gtadoc_decompress(self.handle, tokens.data_ptr(), file_off.data_ptr(), _stream_ptr(stream)))
        return tokens[:T], file_off

    def sort(self, word_counts: torch.Tensor | None = None, stream=None):
        """(ids int32[K], counts int64[K]) device tensors, count desc then id asc."""
        V = self.vocab
        ids = torch.empty(V, dtype=torch.int32, device=self.ctx.device)
        cnt = torch.empty(V, dtype=torch.int64, device=self.ctx.device)
        num = torch.empty(1, dtype=torch.int64, device=self.ctx.device)
        wc = word_counts.data_ptr() if word_counts is not None else None
        _check(lib().gtadoc_sort(self.handle, wc, ids.data_ptr(), cnt.data_ptr(), num.data_ptr(),
                                 _stream_ptr(stream)))
        return ids, cnt, num

    def _result(self, fn, *args, stream=None) -> Result:
        h = _vp()
        _check(fn(self.handle, *args, ctypes.byref(h), _stream_ptr(stream)))
        return _wrap_result(self.ctx, h)


    def term_vector(self, strategy: int | None = None, stream=None) -> Result:
        """Per-file (word, count) rows: arrays (off int64[F+1], word int32[NNZ],
        count int64[NNZ]). strategy: None/TV_AUTO (the selector), TV_BOTTOM_UP
        or TV_TOP_DOWN."""
        if strategy is None:
            return self._result(lib().gtadoc_term_vector, stream=stream)
        return self._result(lib().gtadoc_term_vector_ex, int(strategy), stream=stream)

    def edges(self, stream=None) -> int:
        """E: distinct (parent, child) rule pairs (counted once, then kept)."""
        v = _i64()
        _check(lib().gtadoc_grammar_edges(self.handle, ctypes.byref(v), _stream_ptr(stream)))
        return v.value

    def query_bytes(self, kind: int, n: int = 0, strategy: int = TV_AUTO, stream=None) -> int:
        """Arena bytes a query of this kind takes at its peak (measured on the
        first request by running it once, then kept)."""
        v = _u64()
        _check(lib().gtadoc_query_bytes(self.handle, int(kind), int(n), int(strategy), ctypes.byref(v),
                                        _stream_ptr(stream)))
        return v.value

    def tv_strategy(self) -> int:
        """The traversal the selector (TV_AUTO) takes for this grammar."""
        v = _int()
        _check(lib().gtadoc_term_vector_strategy(self.handle, ctypes.byref(v)))
        return v.value

    def inverted_index(self, stream=None) -> Result:
        return self._result(lib().gtadoc_inverted_index, stream=stream)

    def inverted_index_from(self, term_vector: "Result", stream=None) -> Result:
        """Inverted index from this grammar's term vector result (no recomputation)."""
        return self._result(lib().gtadoc_inverted_index_from_tv, term_vector.handle, stream=stream)

    def ranked_inverted_index(self, stream=None) -> Result:
        """Per word, the files containing it by term frequency descending, then
        file ascending: arrays (off int64[V+1], file int32[NNZ], tf int64[NNZ])."""
        return self._result(lib().gtadoc_ranked_inverted_index, stream=stream)

    def ranked_inverted_index_from(self, term_vector: "Result", stream=None) -> Result:
        """The ranked inverted index from a term vector result of this grammar."""
        return self._result(lib().gtadoc_ranked_inverted_index_from_tv, term_vector.handle, stream=stream)

    def sequence_count_wide(self, n: int, stream=None) -> Result:
        """n-gram counts (n in 2..8) with 126-bit keys: arrays (hi int64[U],
        lo int64[U], count int64[U]), ascending (hi, lo)."""
        return self._result(lib().gtadoc_sequence_count_wide, n, stream=stream)

    def sequence_count(self, n: int, stream=None) -> Result:
        return self._result(lib().gtadoc_sequence_count, n, stream=stream)


def _wrap_result(ctx: Context, h) -> Result:
    """A Result over the arrays of result handle h (views into the arena)."""
    arrays = []
    i = 0
    while True:
        p, n, eb = _vp(), _i64(), _int()
        if lib().gtadoc_result_array(h, i, ctypes.byref(p), ctypes.byref(n), ctypes.byref(eb)) != OK:
            break
        arrays.append(_dev_tensor(p.value or ctx.arena.data_ptr(), n.value, eb.value, ctx.arena))
        i += 1
    return Result(arrays, h, ctx)


class Batch:
    """A batch plan: word counts of many grammars in one launch sequence."""

    def __init__(self, ctx: Context, max_items: int, max_entries: int):
        self.ctx = ctx
        h = _vp()
        _check(lib().gtadoc_batch_create(ctx.handle, int(max_items), int(max_entries), ctypes.byref(h)))
        self.handle = h
        ctx._children.add(self)

    def word_count(self, grammars, outs, stream=None):
        n = len(grammars)
        gs = (ctypes.c_void_p * max(n, 1))(*[g.handle.value for g in grammars])
        os_ = (ctypes.c_void_p * max(n, 1))(*[o.data_ptr() for o in outs])
        _check(lib().gtadoc_batch_word_count(self.handle, gs, os_, n, _stream_ptr(stream)))
        return outs

    def submit(self, queries: list[dict], stream=None) -> list:
        """A mixed batch (gtadoc_batch_submit). Each query is a dict with
        grammar, kind (QUERY_*), and n (sequence count), counts (word count:
        int64 tensor of vocab entries) or strategy (term vector). Returns, per
        query, the counts tensor, a Result, or a GtadocError for a query that
        failed alone."""
        n = len(queries)
        arr = (QueryStruct * max(n, 1))()
        for i, q in enumerate(queries):
            arr[i].grammar = q["grammar"].handle.value
            arr[i].kind = int(q["kind"])
            arr[i].n = int(q.get("n", 0))
            c = q.get("counts")
            arr[i].counts = c.data_ptr() if c is not None else None
            arr[i].strategy = int(q.get("strategy", TV_AUTO))
        _check(lib().gtadoc_batch_submit(self.handle, arr, n, _stream_ptr(stream)))
        out = []
        for i, q in enumerate(queries):
            st = arr[i].status
            if st != OK:
                out.append(GtadocError(st, lib().gtadoc_last_error().decode()))
            elif q["kind"] == QUERY_WORD_COUNT:
                out.append(q["counts"])
            else:
                out.append(_wrap_result(self.ctx, _vp(arr[i].result)))
        return out

    def close(self):
        if self.handle and self.ctx.handle:
            lib().gtadoc_batch_destroy(self.handle)
        self.handle = None

    free = close

    def __del__(self):
        # no HIP call during interpreter shutdown: the runtime (and a
        # profiler's tool library) may already be torn down
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def to_u64(t: torch.Tensor) -> np.ndarray:
    """Host copy of an int64 device tensor holding uint64 values."""
    return t.cpu().numpy().view(np.uint64)
