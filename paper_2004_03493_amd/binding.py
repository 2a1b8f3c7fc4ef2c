"""Thin Python binding of libexactsim.so (argument marshalling only).

Each ``es_*`` function here has the name and meaning of the C entry point in
``include/exactsim.h``; arguments that the C side takes as device pointers
are PyTorch tensors on the context's device, used only as device memory.
Every step of a query runs in the library's HIP kernels.  If the library is
missing, importing this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libexactsim.so")

ES_OK = 0
ES_EINVAL = -1
ES_ERANGE = -2
ES_ENOMEM = -3
ES_EDEVICE = -4
ES_EOVERFLOW = -5
ES_EUNSUPPORTED = -6

ES_ALLOC_PI2 = 0
ES_ALLOC_PI = 1
ES_ALLOC_LEARNED = 2
ES_LDE_OFF, ES_LDE_AS_PRINTED, ES_LDE_REDUCED = 0, 1, 2
ES_LDE_MAX_LEVEL = 3
ES_LEARNED_FLOOR = 0.5  # recommended v_floor_ratio of the learned allocation

ES_DEDUP = 1
ES_DROP_SELF_LOOPS = 2
ES_LEVELS_PULL = 4
ES_LEVELS_BINNED = 8

SYMBOLS = (
    "es_ctx_create", "es_ctx_destroy", "es_ctx_sync", "es_status_str", "es_last_error",
    "es_graph_from_edges", "es_graph_destroy", "es_graph_info", "es_graph_level_pass", "es_graph_degrees",
    "es_num_levels", "es_total_samples", "es_forward", "es_budget", "es_walk_pairs", "es_diag",
    "es_backward", "es_single_source", "es_topk", "es_topk_noalloc", "es_batch", "es_batch_tuning", "es_batch_block_width",
    "es_mlp_num_params", "es_mlp_features", "es_mlp_infer", "es_mlp_grad", "es_mlp_train", "es_mlp_load",
    "es_budget_weighted", "es_lde_plan", "es_walk_pairs_lde", "es_diag_lde",
    "es_forward_sparse", "es_sparse_capacity",
)


class EsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class QueryOpts(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double), ("eps", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("r_scale", ctypes.c_double), ("alloc", ctypes.c_int32), ("exact_small_din", ctypes.c_int32),
                ("d_override", ctypes.c_void_p), ("v_floor_ratio", ctypes.c_double), ("lde", ctypes.c_int32),
                ("sparse_eps", ctypes.c_double), ("lde_max_level", ctypes.c_int32)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("use_hip_graph", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("force_width", ctypes.c_int32), ("force_rows", ctypes.c_int32),
                ("block_width", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("active_nodes", ctypes.c_int32), ("R", ctypes.c_double),
                ("pairs", ctypes.c_uint64), ("pairs_requested", ctypes.c_uint64), ("meets", ctypes.c_uint64),
                ("philox_blocks", ctypes.c_uint64),
                ("walk_steps", ctypes.c_uint64), ("ms_forward", ctypes.c_float),
                ("ms_budget", ctypes.c_float), ("ms_walk", ctypes.c_float), ("ms_diag", ctypes.c_float),
                ("ms_backward", ctypes.c_float), ("lde_source_level", ctypes.c_int32),
                ("lde_source_zsum", ctypes.c_double), ("level_entries", ctypes.c_uint64),
                ("level_bytes", ctypes.c_uint64), ("workspace_bytes", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load_library(path: str = _LIB_PATH) -> ctypes.CDLL:
    """Load libexactsim.so and declare its signatures; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libexactsim.so not built at {path}: run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64, u32, u64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
    sig = {
        "es_ctx_create": [ctypes.c_int, P, ctypes.POINTER(P)],
        "es_ctx_destroy": [P],
        "es_ctx_sync": [P],
        "es_status_str": [ctypes.c_int],
        "es_last_error": [P],
        "es_graph_from_edges": [P, i32, i64, P, P, u32, ctypes.POINTER(P)],
        "es_graph_destroy": [P],
        "es_graph_info": [P, ctypes.POINTER(i32), ctypes.POINTER(i64)],
        "es_graph_level_pass": [P, ctypes.POINTER(i32)],
        "es_graph_degrees": [P, P, P, P],
        "es_num_levels": [dbl, dbl, ctypes.POINTER(i32)],
        "es_total_samples": [i32, dbl, dbl, dbl, ctypes.POINTER(dbl)],
        "es_forward": [P, P, i32, dbl, i32, P, P],
        "es_forward_sparse": [P, P, i32, dbl, i32, dbl, i64, P, P, ctypes.POINTER(u64), P],
        "es_sparse_capacity": [i32, i64, i32, dbl, dbl, ctypes.POINTER(i64)],
        "es_budget": [P, P, P, dbl, i32, i32, P, ctypes.POINTER(u64)],
        "es_walk_pairs": [P, P, P, P, u64, dbl, P],
        "es_diag": [P, P, P, P, dbl, i32, P],
        "es_backward": [P, P, P, i32, P, dbl, P],
        "es_single_source": [P, P, i32, ctypes.POINTER(QueryOpts), P, ctypes.POINTER(Stats)],
        "es_topk": [P, P, i32, i32, i32, P, P],
        "es_topk_noalloc": [P, P, i32, i32, i32, P, P],
        "es_batch": [P, P, i32, P, P, i32, ctypes.POINTER(QueryOpts), ctypes.POINTER(BatchOpts), P,
                     ctypes.POINTER(Stats)],
        "es_batch_tuning": [P, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "es_batch_block_width": [P, i32, ctypes.POINTER(i32)],
        "es_mlp_num_params": [],
        "es_mlp_features": [P, P, dbl, P],
        "es_mlp_infer": [P, P, P, i64, dbl, P, P],
        "es_mlp_grad": [P, P, P, P, P, i64, dbl, P, ctypes.POINTER(dbl)],
        "es_mlp_train": [P, P, P, P, i64, dbl, i32, ctypes.c_float, P, P],
        "es_mlp_load": [P, P],
        "es_budget_weighted": [P, P, P, P, dbl, i32, dbl, P],
        "es_lde_plan": [P, P, P, dbl, i32, i32, P, P, P],
        "es_walk_pairs_lde": [P, P, P, P, P, u64, dbl, P],
        "es_diag_lde": [P, P, P, P, P, P, dbl, i32, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.es_status_str.restype = ctypes.c_char_p
    lib.es_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int, ctx=None):
    if status != ES_OK:
        lib = load_library()
        msg = lib.es_status_str(status).decode()
        if ctx is not None and getattr(ctx, "handle", None):
            detail = lib.es_last_error(ctx.handle).decode()
            if detail:
                msg = f"{msg}: {detail}"
        raise EsError(status, msg)


def _ptr(t, dtype, numel=None, name="tensor"):
    """Device pointer of a contiguous tensor of the given dtype (None -> NULL)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name}: must live in device memory")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name}: needs at least {numel} elements, has {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """es_ctx on a HIP device, enqueueing on the current PyTorch stream."""

    def __init__(self, device: int = 0, stream=None):
        lib = load_library()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib.es_ctx_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            load_library().es_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self):
        _check(load_library().es_ctx_sync(self.handle), self)


class Graph:
    """es_graph built from host int32 edge arrays."""

    def __init__(self, ctx: Context, n: int, src, dst, flags: int = ES_DEDUP | ES_DROP_SELF_LOOPS):
        import numpy as np
        lib = load_library()
        src = np.ascontiguousarray(src, dtype=np.int32)
        dst = np.ascontiguousarray(dst, dtype=np.int32)
        if src.shape != dst.shape:
            raise ValueError("src and dst differ in length")
        h = ctypes.c_void_p()
        _check(lib.es_graph_from_edges(ctx.handle, n, len(src), src.ctypes.data, dst.ctypes.data, flags,
                                       ctypes.byref(h)), ctx)
        self.ctx = ctx
        self.handle = h
        nn = ctypes.c_int32()
        mm = ctypes.c_int64()
        _check(lib.es_graph_info(h, ctypes.byref(nn), ctypes.byref(mm)), ctx)
        self.n = nn.value
        self.m = mm.value
        binned = ctypes.c_int32()
        _check(lib.es_graph_level_pass(h, ctypes.byref(binned)), ctx)
        self.binned = bool(binned.value)

    def close(self):
        if self.handle:
            load_library().es_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def es_num_levels(c: float, eps: float) -> int:
    L = ctypes.c_int32()
    _check(load_library().es_num_levels(c, eps, ctypes.byref(L)))
    return L.value


def es_total_samples(n: int, c: float, eps: float, r_scale: float = 1.0) -> float:
    R = ctypes.c_double()
    _check(load_library().es_total_samples(n, c, eps, r_scale, ctypes.byref(R)))
    return R.value


def es_graph_degrees(ctx: Context, g: Graph, din=None, dout=None):
    _check(load_library().es_graph_degrees(ctx.handle, g.handle, _ptr(din, torch.int32, g.n, "din"),
                                           _ptr(dout, torch.int32, g.n, "dout")), ctx)


def es_forward(ctx: Context, g: Graph, u: int, c: float, L: int, levels, pi):
    _check(load_library().es_forward(ctx.handle, g.handle, u, c, L,
                                     _ptr(levels, torch.float64, (L + 1) * g.n, "levels"),
                                     _ptr(pi, torch.float64, g.n, "pi")), ctx)


def es_sparse_capacity(n: int, m: int, L: int, c: float, sparse_eps: float) -> int:
    cap = ctypes.c_int64()
    _check(load_library().es_sparse_capacity(n, m, L, c, sparse_eps, ctypes.byref(cap)))
    return cap.value


def es_forward_sparse(ctx: Context, g: Graph, u: int, c: float, L: int, sparse_eps: float, idx, val, pi=None):
    """Kept entries of the levels (sparse linearization); returns the count per level."""
    cap = min(idx.numel(), val.numel())
    counts = (ctypes.c_uint64 * (L + 1))()
    _check(load_library().es_forward_sparse(ctx.handle, g.handle, u, c, L, sparse_eps, cap,
                                            _ptr(idx, torch.int32, cap, "idx"), _ptr(val, torch.float64, cap, "val"),
                                            counts, _ptr(pi, torch.float64, g.n, "pi")), ctx)
    return [int(x) for x in counts]


def es_budget(ctx: Context, g: Graph, pi, R: float, alloc: int, exact_small_din: bool, Rk,
              want_total: bool = False):
    tot = ctypes.c_uint64()
    _check(load_library().es_budget(ctx.handle, g.handle, _ptr(pi, torch.float64, g.n, "pi"), R, alloc,
                                    int(exact_small_din), _ptr(Rk, torch.uint64, g.n, "Rk"),
                                    ctypes.byref(tot) if want_total else None), ctx)
    return tot.value if want_total else None


def es_walk_pairs(ctx: Context, g: Graph, r_begin, r_end, seed: int, c: float, M):
    _check(load_library().es_walk_pairs(ctx.handle, g.handle, _ptr(r_begin, torch.uint64, g.n, "r_begin"),
                                        _ptr(r_end, torch.uint64, g.n, "r_end"), seed, c,
                                        _ptr(M, torch.uint64, g.n, "M")), ctx)


def es_diag(ctx: Context, g: Graph, Rk, M, c: float, exact_small_din: bool, D):
    _check(load_library().es_diag(ctx.handle, g.handle, _ptr(Rk, torch.uint64, g.n, "Rk"),
                                  _ptr(M, torch.uint64, g.n, "M"), c, int(exact_small_din),
                                  _ptr(D, torch.float64, g.n, "D")), ctx)


def es_backward(ctx: Context, g: Graph, levels, L: int, D, c: float, s):
    _check(load_library().es_backward(ctx.handle, g.handle, _ptr(levels, torch.float64, (L + 1) * g.n, "levels"),
                                      L, _ptr(D, torch.float64, g.n, "D"), c,
                                      _ptr(s, torch.float64, g.n, "s")), ctx)


def make_opts(c: float, eps: float, seed: int, r_scale: float = 1.0, alloc: int = ES_ALLOC_PI2,
              exact_small_din: bool = True, d_override=None, v_floor_ratio: float = ES_LEARNED_FLOOR,
              lde: int = ES_LDE_OFF, sparse_eps: float = 0.0, lde_max_level: int = ES_LDE_MAX_LEVEL) -> QueryOpts:
    o = QueryOpts()
    o.c, o.eps, o.seed, o.r_scale = c, eps, seed, r_scale
    o.alloc, o.exact_small_din = alloc, int(exact_small_din)
    o.d_override = None if d_override is None else d_override.data_ptr()
    o.v_floor_ratio = v_floor_ratio
    o.lde = lde
    o.sparse_eps = sparse_eps
    o.lde_max_level = lde_max_level
    return o


def es_single_source(ctx: Context, g: Graph, u: int, opts: QueryOpts, s_out, want_stats: bool = True):
    if opts.d_override:
        pass  # pointer already taken from a device tensor by make_opts
    st = Stats()
    _check(load_library().es_single_source(ctx.handle, g.handle, u, ctypes.byref(opts),
                                           _ptr(s_out, torch.float64, g.n, "s_out"),
                                           ctypes.byref(st) if want_stats else None), ctx)
    return st if want_stats else None


def es_topk(ctx: Context, s, n: int, exclude: int, k: int, idx_out, val_out=None):
    _check(load_library().es_topk(ctx.handle, _ptr(s, torch.float64, n, "s"), n, exclude, k,
                                  _ptr(idx_out, torch.int32, k, "idx_out"),
                                  _ptr(val_out, torch.float64, k, "val_out")), ctx)


def es_topk_noalloc(ctx: Context, s, n: int, exclude: int, k: int, idx_out, val_out=None):
    _check(load_library().es_topk_noalloc(ctx.handle, _ptr(s, torch.float64, n, "s"), n, exclude, k,
                                          _ptr(idx_out, torch.int32, k, "idx_out"),
                                          _ptr(val_out, torch.float64, k, "val_out")), ctx)


def es_batch(ctx: Context, graphs, graph_of_query, sources, opts: QueryOpts, outs, use_hip_graph: bool = False,
             autotune: bool = True, force_width: int = 0, force_rows: int = 0, want_stats: bool = True,
             block_width: int = 0):
    """Batched queries: graphs is a list of Graph, outs a list of float64 device tensors."""
    import numpy as np
    lib = load_library()
    nq = len(sources)
    if len(graph_of_query) != nq or len(outs) != nq:
        raise ValueError("graph_of_query, sources and outs must have one entry per query")
    gh = (ctypes.c_void_p * len(graphs))(*[g.handle.value for g in graphs])
    goq = np.ascontiguousarray(graph_of_query, dtype=np.int32)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    ptrs = []
    for q in range(nq):
        gi = int(goq[q])
        n = graphs[gi].n if 0 <= gi < len(graphs) else None  # a bad index is the library's to report
        ptrs.append(_ptr(outs[q], torch.float64, n, f"outs[{q}]").value)
    op = (ctypes.c_void_p * nq)(*ptrs)
    bo = BatchOpts(int(use_hip_graph), int(autotune), int(force_width), int(force_rows), int(block_width))
    st = Stats()
    _check(lib.es_batch(ctx.handle, gh, len(graphs), goq.ctypes.data, src.ctypes.data, nq, ctypes.byref(opts),
                        ctypes.byref(bo), op, ctypes.byref(st) if want_stats else None), ctx)
    return st if want_stats else None


def es_batch_tuning(g: Graph, B: int):
    w = ctypes.c_int32()
    r = ctypes.c_int32()
    _check(load_library().es_batch_tuning(g.handle, B, ctypes.byref(w), ctypes.byref(r)))
    return w.value, r.value


def es_batch_block_width(g: Graph, S: int) -> int:
    w = ctypes.c_int32()
    _check(load_library().es_batch_block_width(g.handle, S, ctypes.byref(w)))
    return w.value


def es_mlp_num_params() -> int:
    return int(load_library().es_mlp_num_params())


def es_mlp_features(ctx: Context, g: Graph, c: float, feats):
    _check(load_library().es_mlp_features(ctx.handle, g.handle, c, _ptr(feats, torch.float32, 6 * g.n, "feats")),
           ctx)


def es_mlp_infer(ctx: Context, weights, feats, N: int, c: float, p_out=None, v_out=None):
    _check(load_library().es_mlp_infer(ctx.handle, _ptr(weights, torch.float32, es_mlp_num_params(), "weights"),
                                       _ptr(feats, torch.float32, 6 * N, "feats"), N, c,
                                       _ptr(p_out, torch.float32, N, "p_out"), _ptr(v_out, torch.float32, N, "v_out")),
           ctx)


def es_mlp_grad(ctx: Context, weights, feats, R, M, N: int, c: float, grad) -> float:
    loss = ctypes.c_double()
    _check(load_library().es_mlp_grad(ctx.handle, _ptr(weights, torch.float32, es_mlp_num_params(), "weights"),
                                      _ptr(feats, torch.float32, 6 * N, "feats"), _ptr(R, torch.uint64, N, "R"),
                                      _ptr(M, torch.uint64, N, "M"), N, c,
                                      _ptr(grad, torch.float32, es_mlp_num_params(), "grad"), ctypes.byref(loss)), ctx)
    return loss.value


def es_mlp_train(ctx: Context, feats, R, M, N: int, c: float, epochs: int, lr: float, weights):
    import numpy as np
    losses = np.zeros(epochs, dtype=np.float32)
    _check(load_library().es_mlp_train(ctx.handle, _ptr(feats, torch.float32, 6 * N, "feats"),
                                       _ptr(R, torch.uint64, N, "R"), _ptr(M, torch.uint64, N, "M"), N, c, epochs,
                                       lr, _ptr(weights, torch.float32, es_mlp_num_params(), "weights"),
                                       losses.ctypes.data), ctx)
    return losses


def es_mlp_load(ctx: Context, weights):
    _check(load_library().es_mlp_load(ctx.handle, _ptr(weights, torch.float32, es_mlp_num_params(), "weights")),
           ctx)


def es_budget_weighted(ctx: Context, g: Graph, pi, v, R: float, exact_small_din: bool, floor_ratio: float, Rk):
    _check(load_library().es_budget_weighted(ctx.handle, g.handle, _ptr(pi, torch.float64, g.n, "pi"),
                                             _ptr(v, torch.float32, g.n, "v"), R, int(exact_small_din), floor_ratio,
                                             _ptr(Rk, torch.uint64, g.n, "Rk")), ctx)


def es_lde_plan(ctx: Context, g: Graph, Rk, c: float, mode: int, max_level: int, ell, zsum, Rk_out):
    _check(load_library().es_lde_plan(ctx.handle, g.handle, _ptr(Rk, torch.uint64, g.n, "Rk"), c, mode, max_level,
                                      _ptr(ell, torch.int32, g.n, "ell"), _ptr(zsum, torch.float64, g.n, "zsum"),
                                      _ptr(Rk_out, torch.uint64, g.n, "Rk_out")), ctx)


def es_walk_pairs_lde(ctx: Context, g: Graph, r_begin, r_end, ell, seed: int, c: float, M):
    _check(load_library().es_walk_pairs_lde(ctx.handle, g.handle, _ptr(r_begin, torch.uint64, g.n, "r_begin"),
                                            _ptr(r_end, torch.uint64, g.n, "r_end"),
                                            _ptr(ell, torch.int32, g.n, "ell"), seed, c,
                                            _ptr(M, torch.uint64, g.n, "M")), ctx)


def es_diag_lde(ctx: Context, g: Graph, Rk, M, ell, zsum, c: float, exact_small_din: bool, D):
    _check(load_library().es_diag_lde(ctx.handle, g.handle, _ptr(Rk, torch.uint64, g.n, "Rk"),
                                      _ptr(M, torch.uint64, g.n, "M"), _ptr(ell, torch.int32, g.n, "ell"),
                                      _ptr(zsum, torch.float64, g.n, "zsum"), c, int(exact_small_din),
                                      _ptr(D, torch.float64, g.n, "D")), ctx)
