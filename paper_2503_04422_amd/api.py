"""Python binding of libpdx: argument marshalling only.

Each function has the name of the C entry point it calls.  Tensors must be
CUDA (HIP) tensors; torch provides the device memory (index buffers,
workspaces, outputs) and the current stream.  Every step of the search runs
in the library's HIP kernels.

``stream=``: when a stream is given, the call's own allocations and copies
(workspace, outputs, contiguous copies of the inputs) are made with that
stream current, so torch's caching allocator ties them to the stream the
library's kernels run on and cannot hand their memory to other work while
those kernels still read it; the searches also record the index memory on
the stream.  Inputs the caller made on another stream must be ordered
before the call by the caller, as with any torch op.
"""
from __future__ import annotations

import contextlib
import ctypes
import functools
import inspect
import math
from typing import Optional, Tuple

import torch

from . import _lib
from ._lib import check, lib


def _stream(stream: Optional[torch.cuda.Stream]) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _on_stream(fn):
    """Run ``fn`` with its ``stream`` argument (if given) as torch's current
    stream, so every tensor the call allocates or copies belongs to the
    stream the library's kernels are queued on."""
    sig = inspect.signature(fn)

    @functools.wraps(fn)
    def wrapped(*args, **kwargs):
        stream = sig.bind_partial(*args, **kwargs).arguments.get("stream")
        ctx = torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()
        with ctx:
            return fn(*args, **kwargs)

    return wrapped


def _hold_index(index: "PdxIndex") -> None:
    """The index memory stays reserved until the current stream's queued
    work (this call's kernels) is done, even if the index is dropped."""
    index.mem.record_stream(torch.cuda.current_stream(index.mem.device))


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _dev_f32(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != torch.float32 or t.dim() != 2:
        raise TypeError(f"{name} must be a 2-D float32 tensor")
    return t.contiguous()


_MODES = {"linear": _lib.PDX_MODE_LINEAR, "bond": _lib.PDX_MODE_BOND}
_BOUNDS = {"ads": 0, "bond": 1, "zones": 2, "bsa": 3}
_DTYPES = {"f32": _lib.PDX_DTYPE_F32, "bf16": _lib.PDX_DTYPE_BF16, "fp8": _lib.PDX_DTYPE_FP8}


class PdxIndex:
    """Host handle plus the device buffer it points into."""

    def __init__(self, handle: ctypes.c_void_p, mem: torch.Tensor, n: int, d: int, kind: str,
                 nlist: int = 0, dtype: str = "f32"):
        self._h = handle
        self.mem = mem
        self.n = n
        self.d = d
        self.kind = kind
        self.nlist = nlist
        self.dtype = dtype

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib.pdx_free(h)
            self._h = ctypes.c_void_p(None)


@_on_stream
def pdx_build(x: torch.Tensor, start_rows: int = 0,
              stream: Optional[torch.cuda.Stream] = None) -> PdxIndex:
    """Flat PDX index of the rows of ``x`` ([n, d] float32 on the GPU)."""
    x = _dev_f32(x, "x")
    n, d = x.shape
    params = _lib.pdx_build_params(0, int(start_rows))
    nbytes = lib.pdx_build_bytes(n, d, ctypes.byref(params))
    if nbytes == 0:
        raise ValueError(f"unsupported shape n={n} d={d}")
    mem = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    h = ctypes.c_void_p()
    st = lib.pdx_build(_ptr(x), n, d, ctypes.byref(params), _ptr(mem), nbytes, _stream(stream),
                       ctypes.byref(h))
    check(st, "pdx_build")
    return PdxIndex(h, mem, n, d, "flat")


_METRICS = {"l2": _lib.PDX_METRIC_L2, "l1": _lib.PDX_METRIC_L1, "ip": _lib.PDX_METRIC_IP}


def pdx_search_exact_workspace(index: PdxIndex, nq: int, k: int, mode: str = "bond", chunk: int = 0,
                               tile_groups: int = 0, queries_per_block: int = 0, metric: str = "l2",
                               start_rows: int = 0, rounds: int = 0, dense_min: int = 0) -> int:
    p = _lib.pdx_search_params(_MODES[mode], chunk, tile_groups, queries_per_block, None, None, _METRICS[metric],
                               int(start_rows), None, int(rounds), int(dense_min))
    return int(lib.pdx_search_exact_workspace(index.handle, nq, k, ctypes.byref(p)))


@_on_stream
def pdx_search_exact(index: PdxIndex, q: torch.Tensor, k: int, mode: str = "bond", chunk: int = 0,
                     tile_groups: int = 0, queries_per_block: int = 0,
                     workspace: Optional[torch.Tensor] = None,
                     phase_events=None, counters: Optional[torch.Tensor] = None,
                     out: Optional[Tuple[torch.Tensor, torch.Tensor]] = None, metric: str = "l2",
                     start_rows: int = 0, chunk_survivors: Optional[torch.Tensor] = None,
                     rounds: int = 0, dense_min: int = 0,
                     stream: Optional[torch.cuda.Stream] = None) -> Tuple[torch.Tensor, torch.Tensor]:
    """Exact k nearest neighbours; returns (ids [nq, k] int64, dist [nq, k] float32).

    ``metric``: "l2" (squared Euclidean), "l1" (sum of absolute
    differences) or "ip" (-q.v, mode "linear" only).
    ``start_rows``: bucket layout, rows of the nearest bucket START scans
    (0 = 128).
    ``rounds``, ``dense_min``: tile-scan schedule (0 = defaults: rounds 2 on
    the bucket layout and 4 on the flat one, dense_min 4;
    pdx_exact_tune picks them); the result does not depend on them.
    ``phase_events``: optional ctypes array of 4 hipEvent_t handles;
    ``counters``: optional int64 GPU tensor of 4 value counters;
    ``chunk_survivors``: optional int64 GPU tensor of ceil(D / chunk)
    per-chunk survivor counts of the pruned scan (added to)."""
    q = _dev_f32(q, "q")
    nq = q.shape[0]
    if q.shape[1] != index.d:
        raise ValueError("query dimension does not match the index")
    p = _lib.pdx_search_params(_MODES[mode], chunk, tile_groups, queries_per_block,
                               ctypes.cast(phase_events, ctypes.c_void_p) if phase_events is not None else None,
                               _ptr(counters), _METRICS[metric], int(start_rows), _ptr(chunk_survivors),
                               int(rounds), int(dense_min))
    if out is None:
        ids = torch.empty((nq, k), dtype=torch.int64, device=q.device)
        dist = torch.empty((nq, k), dtype=torch.float32, device=q.device)
    else:
        ids, dist = out
    need = lib.pdx_search_exact_workspace(index.handle, nq, k, ctypes.byref(p))
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=q.device)
    _hold_index(index)
    st = lib.pdx_search_exact(index.handle, _ptr(q), nq, k, ctypes.byref(p), _ptr(workspace),
                              workspace.numel(), _ptr(ids), _ptr(dist), _stream(stream))
    check(st, "pdx_search_exact")
    return ids, dist


_ORDERS = {"natural": _lib.PDX_ORDER_NATURAL, "bond": _lib.PDX_ORDER_BOND, "zones": _lib.PDX_ORDER_ZONES}


@_on_stream
def pdx_query_order(index: PdxIndex, q: torch.Tensor, order: str = "bond", tile_offsets: bool = False,
                    stream: Optional[torch.cuda.Stream] = None):
    """The dimension visit order the searches use for each query
    (pdx_query_order): (perm [nq, d] int32, qval [nq, d] float32, off
    [nq, d] int16 holding the uint16 LDS tile offsets, or None)."""
    q = _dev_f32(q, "q")
    nq = q.shape[0]
    if q.shape[1] != index.d:
        raise ValueError("query dimension does not match the index")
    perm = torch.empty((nq, index.d), dtype=torch.int32, device=q.device)
    qval = torch.empty((nq, index.d), dtype=torch.float32, device=q.device)
    off = torch.empty((nq, index.d), dtype=torch.int16, device=q.device) if tile_offsets else None
    need = lib.pdx_query_order_workspace(index.handle, nq)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=q.device)
    _hold_index(index)
    check(lib.pdx_query_order(index.handle, _ptr(q), nq, _ORDERS[order], _ptr(perm), _ptr(qval), _ptr(off),
                              _ptr(ws), ws.numel(), _stream(stream)), "pdx_query_order")
    return perm, qval, off


@_on_stream
def pdx_ivf_build(x: torch.Tensor, nlist: int, gaussian: Optional[torch.Tensor],
                  init_rows: Optional[torch.Tensor], kmeans_iters: int = 0, lowp: Tuple[str, ...] = (),
                  rotation: Optional[torch.Tensor] = None, centroids: Optional[torch.Tensor] = None,
                  assign: Optional[torch.Tensor] = None, rotation_kind: str = "random", pca_iters: int = 0,
                  stream: Optional[torch.cuda.Stream] = None) -> PdxIndex:
    """IVF index over rotated rows; buckets stored as PDX groups.
    rotation_kind "random": the Q of the QR of ``gaussian`` (no rotation
    when it is None); "pca": the rows' principal directions, largest
    variance first (``gaussian`` unused); a given ``rotation`` overrides
    both."""
    x = _dev_f32(x, "x")
    n, d = x.shape
    keep = [t.contiguous() if t is not None else None for t in (gaussian, init_rows, rotation, centroids, assign)]
    g, ir, rot, cen, asg = keep
    if g is not None and g.dtype != torch.float64:
        raise TypeError("gaussian must be float64")
    if ir is not None and ir.dtype != torch.int64:
        raise TypeError("init_rows must be int64")
    if asg is not None and asg.dtype != torch.int32:
        raise TypeError("assign must be int32")
    mask = 0
    for name in lowp:
        if name not in ("bf16", "fp8"):
            raise ValueError(f"unknown low-precision storage {name!r}")
        mask |= 1 << _DTYPES[name]
    kinds = {"random": _lib.PDX_ROTATION_RANDOM, "pca": _lib.PDX_ROTATION_PCA}
    if rotation_kind not in kinds:
        raise ValueError(f"unknown rotation_kind {rotation_kind!r}")
    p = _lib.pdx_ivf_params(int(kmeans_iters), mask, _ptr(g), _ptr(ir), _ptr(rot), _ptr(cen), _ptr(asg),
                            kinds[rotation_kind], int(pca_iters))
    nbytes = lib.pdx_ivf_build_bytes(n, d, nlist, ctypes.byref(p))
    if nbytes == 0:
        raise ValueError(f"unsupported IVF shape n={n} d={d} nlist={nlist}")
    mem = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    h = ctypes.c_void_p()
    st = lib.pdx_ivf_build(_ptr(x), n, d, nlist, ctypes.byref(p), _ptr(mem), nbytes, _stream(stream),
                           ctypes.byref(h))
    check(st, "pdx_ivf_build")
    return PdxIndex(h, mem, n, d, "ivf", nlist, "+".join(("f32",) + tuple(lowp)))


@_on_stream
def pdx_ivf_export(index: PdxIndex, stream: Optional[torch.cuda.Stream] = None):
    """(rotation [d,d], centroids [nlist,d], assign [n] int32, list_sizes [nlist] int32)."""
    dev = index.mem.device
    rot = torch.empty((index.d, index.d), dtype=torch.float32, device=dev)
    cen = torch.empty((index.nlist, index.d), dtype=torch.float32, device=dev)
    asg = torch.empty(index.n, dtype=torch.int32, device=dev)
    sizes = torch.empty(index.nlist, dtype=torch.int32, device=dev)
    st = lib.pdx_ivf_export(index.handle, _ptr(rot), _ptr(cen), _ptr(asg), _ptr(sizes), _stream(stream))
    check(st, "pdx_ivf_export")
    return rot, cen, asg, sizes


def ivf_test_points(d: int, delta_d: int = 0) -> int:
    """Prune-test points per bucket, C = ceil(D / delta_d) - 1 (the tests
    after c1 = (c + 1) delta_d < D dimensions); delta_d 0 = the library's
    default (32, or D/4 when D < 128)."""
    dd = delta_d if delta_d > 0 else (32 if d >= 128 else max(d // 4, 1))
    return (d + dd - 1) // dd - 1 if dd < d else 0


def pdx_search_ivf_workspace(index: PdxIndex, nq: int, k: int, nprobe: int, delta_d: int = 0,
                             dtype: str = "f32", rerank: int = 0, queries_per_wave: int = 0,
                             engine: int = 0, mlp: Optional["MlpState"] = None, bucket_split: int = 0,
                             bound: str = "ads", prune_mlp: Optional["MlpState"] = None,
                             prune_trace: bool = False, bsa_m: float = 0.0, rerank_capacity: int = 0) -> int:
    """Workspace bytes of pdx_search_ivf with the same arguments (the
    learned stop adds stages, and so item padding; the prune multipliers
    and their traces add per-query tables)."""
    p = _lib.pdx_ivf_search_params(2.1, int(delta_d), _DTYPES[dtype], int(rerank), None, None,
                                   None if mlp is None else _ptr(mlp.mem), 0.5, None, None,
                                   int(queries_per_wave), 0, int(engine), int(bucket_split), _BOUNDS[bound],
                                   None if prune_mlp is None else _ptr(prune_mlp.mem), 1.0, None,
                                   1 if prune_trace else None, 1 if prune_trace else None, 0, float(bsa_m),
                                   int(rerank_capacity))
    return int(lib.pdx_search_ivf_workspace(index.handle, nq, k, nprobe, ctypes.byref(p)))


_LOSSES = {"bce": _lib.PDX_LOSS_BCE, "pinball": _lib.PDX_LOSS_PINBALL}


class MlpState:
    """Device state of one of the search's networks (pdx_mlp_*): the probe
    budget (weighted cross-entropy, kind "bce", w = the negatives' weight)
    or the prune bound (kind "pinball", w = the quantile level)."""

    @_on_stream
    def __init__(self, theta0: torch.Tensor, stream: Optional[torch.cuda.Stream] = None):
        if not theta0.is_cuda or theta0.dtype != torch.float32 or theta0.numel() != _lib.MLP_PARAMS:
            raise TypeError(f"theta0 must be a float32 GPU tensor of {_lib.MLP_PARAMS} values")
        self.mem = torch.empty(lib.pdx_mlp_bytes(), dtype=torch.uint8, device=theta0.device)
        self._ws = None
        check(lib.pdx_mlp_init(_ptr(self.mem), _ptr(theta0.contiguous()), _stream(stream)), "pdx_mlp_init")

    def _workspace(self, n: int) -> torch.Tensor:
        need = lib.pdx_mlp_workspace(n)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.mem.device)
        return self._ws

    @_on_stream
    def forward(self, x: torch.Tensor, stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
        x = _dev_f32(x, "x")
        z = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        check(lib.pdx_mlp_forward(_ptr(self.mem), _ptr(x), x.shape[0], _ptr(z), _stream(stream)), "pdx_mlp_forward")
        return z

    @_on_stream
    def grad(self, x: torch.Tensor, y: torch.Tensor, w: float, kind: str = "bce",
             stream: Optional[torch.cuda.Stream] = None):
        x = _dev_f32(x, "x")
        y = y.contiguous()
        g = torch.empty(_lib.MLP_PARAMS, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        ws = self._workspace(x.shape[0])
        check(lib.pdx_mlp_grad(_ptr(self.mem), _ptr(x), _ptr(y), x.shape[0], _LOSSES[kind], float(w), _ptr(ws),
                               ws.numel(), _ptr(g), _ptr(loss), _stream(stream)), "pdx_mlp_grad")
        return g, loss

    @_on_stream
    def theta(self, stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
        """The float32 parameters [8960] (a copy)."""
        t = torch.empty(_lib.MLP_PARAMS, dtype=torch.float32, device=self.mem.device)
        check(lib.pdx_mlp_export(_ptr(self.mem), _ptr(t), _stream(stream)), "pdx_mlp_export")
        return t

    @_on_stream
    def train_step(self, x: torch.Tensor, y: torch.Tensor, w: float, lr: float, step: int,
                   loss: Optional[torch.Tensor] = None, kind: str = "bce",
                   stream: Optional[torch.cuda.Stream] = None) -> None:
        x = _dev_f32(x, "x")
        ws = self._workspace(x.shape[0])
        check(lib.pdx_mlp_train_step(_ptr(self.mem), _ptr(x), _ptr(y.contiguous()), x.shape[0], _LOSSES[kind],
                                     float(w), float(lr), int(step), _ptr(ws), ws.numel(), _ptr(loss),
                                     _stream(stream)), "pdx_mlp_train_step")


@_on_stream
def pdx_search_ivf(index: PdxIndex, q: torch.Tensor, k: int, nprobe: int, eps0: float = 2.1,
                   delta_d: int = 0, dtype: str = "f32", rerank: int = 0,
                   workspace: Optional[torch.Tensor] = None, phase_events=None,
                   counters: Optional[torch.Tensor] = None, mlp: Optional[MlpState] = None,
                   mlp_threshold: float = 0.5, trace: Optional[Tuple[torch.Tensor, torch.Tensor]] = None,
                   queries_per_wave: int = 0, bucket_order: int = 0, engine: int = 0, bucket_split: int = 0,
                   bound: str = "ads", prune_mlp: Optional[MlpState] = None, prune_scale: float = 1.0,
                   prune_table: Optional[torch.Tensor] = None,
                   prune_trace: Optional[Tuple[torch.Tensor, torch.Tensor]] = None, zone_rows: int = 0,
                   bsa_m: float = 0.0, rerank_capacity: int = 0,
                   stream: Optional[torch.cuda.Stream] = None) -> Tuple[torch.Tensor, torch.Tensor]:
    """Approximate k nearest neighbours (IVF + ADSampling; bound "bond" or
    "zones": PDX-BOND in per-dimension or dimension-zone order, exact within
    the probed buckets, zone_rows the survivor count at or below which
    zones are read from the row-major copy; bound "bsa": BSA's
    Cauchy-Schwarz test with multiplier bsa_m, exact at 1), optionally with the
    learned probe budget (mlp) or recording its training traces
    (trace = (features [nq, nprobe, 72] float32, need [nq] int32)), and
    with the learned prune bound (prune_mlp, prune_scale; prune_table
    receives the multipliers [nq, nprobe - 1, C], C = ivf_test_points(D,
    delta_d)) or recording its traces (prune_trace = (features [nq, k, 72],
    target [nq, k]) float32).  dtype "bf16"/"fp8": the rerank best by the
    scanned distance re-ranked in f32 (rerank > 64: through a per-query
    candidate buffer of rerank_capacity keys, 0 = the library's default)."""
    q = _dev_f32(q, "q")
    nq = q.shape[0]
    if q.shape[1] != index.d:
        raise ValueError("query dimension does not match the index")
    tf, ti = (None, None) if trace is None else trace
    if tf is not None and (tf.dtype != torch.float32 or tf.numel() != nq * nprobe * _lib.MLP_IN
                           or not tf.is_contiguous()):
        raise TypeError("trace features must be contiguous float32 [nq, nprobe, 72]")
    if ti is not None and (ti.dtype != torch.int32 or ti.numel() != nq or not ti.is_contiguous()):
        raise TypeError("trace need must be contiguous int32 [nq]")
    npt = ivf_test_points(index.d, delta_d)
    if prune_table is not None and (prune_table.dtype != torch.float32 or not prune_table.is_contiguous()
                                    or prune_table.numel() != nq * max(nprobe - 1, 0) * npt):
        raise TypeError(f"prune_table must be contiguous float32 [nq, nprobe - 1, {npt}]")
    pf, pt = (None, None) if prune_trace is None else prune_trace
    if pf is not None and (pf.dtype != torch.float32 or not pf.is_contiguous() or pf.numel() != nq * k * _lib.MLP_IN):
        raise TypeError("prune trace features must be contiguous float32 [nq, k, 72]")
    if pt is not None and (pt.dtype != torch.float32 or not pt.is_contiguous() or pt.numel() != nq * k):
        raise TypeError("prune trace targets must be contiguous float32 [nq, k]")
    p = _lib.pdx_ivf_search_params(float(eps0) if math.isfinite(eps0) else float("inf"), int(delta_d),
                                   _DTYPES[dtype], int(rerank),
                                   ctypes.cast(phase_events, ctypes.c_void_p) if phase_events is not None else None,
                                   _ptr(counters), None if mlp is None else _ptr(mlp.mem), float(mlp_threshold),
                                   _ptr(tf), _ptr(ti), int(queries_per_wave), int(bucket_order), int(engine),
                                   int(bucket_split), _BOUNDS[bound],
                                   None if prune_mlp is None else _ptr(prune_mlp.mem), float(prune_scale),
                                   _ptr(prune_table), _ptr(pf), _ptr(pt), int(zone_rows), float(bsa_m),
                                   int(rerank_capacity))
    ids = torch.empty((nq, k), dtype=torch.int64, device=q.device)
    dist = torch.empty((nq, k), dtype=torch.float32, device=q.device)
    need = lib.pdx_search_ivf_workspace(index.handle, nq, k, nprobe, ctypes.byref(p))
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=q.device)
    _hold_index(index)
    st = lib.pdx_search_ivf(index.handle, _ptr(q), nq, k, nprobe, ctypes.byref(p), _ptr(workspace),
                            workspace.numel(), _ptr(ids), _ptr(dist), _stream(stream))
    check(st, "pdx_search_ivf")
    return ids, dist


@_on_stream
def pdx_ivf_tune(index: PdxIndex, q: torch.Tensor, k: int, nprobe: int, eps0: float = 2.1, delta_d: int = 0,
                 dtype: str = "f32", rerank: int = 0, tune_delta_d: bool = True, reps: int = 3,
                 bound: str = "ads", bsa_m: float = 0.0,
                 stream: Optional[torch.cuda.Stream] = None):
    """Fastest scan schedule for this workload (pdx_ivf_tune).  Returns
    (schedule, table): schedule = keyword arguments for pdx_search_ivf
    (engine, queries_per_wave, bucket_order, delta_d); table = every
    candidate with its best time in ms (-1: skipped)."""
    q = _dev_f32(q, "q")
    nq = q.shape[0]
    p = _lib.pdx_ivf_search_params(float(eps0) if math.isfinite(eps0) else float("inf"), int(delta_d),
                                   _DTYPES[dtype], int(rerank), None, None, None, 0.5, None, None, 0, 0, 0, 0,
                                   _BOUNDS[bound], None, 1.0, None, None, None, 0, float(bsa_m), 0)
    need = lib.pdx_ivf_tune_workspace(index.handle, nq, k, nprobe, ctypes.byref(p))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=q.device)
    table = (_lib.pdx_ivf_schedule * _lib.TUNE_CANDIDATES)()
    _hold_index(index)
    st = lib.pdx_ivf_tune(index.handle, _ptr(q), nq, k, nprobe, ctypes.byref(p), int(bool(tune_delta_d)), int(reps),
                          table, _ptr(ws), ws.numel(), _stream(stream))
    check(st, "pdx_ivf_tune")
    sched = {"engine": p.engine, "queries_per_wave": p.queries_per_wave, "bucket_order": p.bucket_order,
             "delta_d": p.delta_d}
    rows = [{"engine": t.engine, "queries_per_wave": t.queries_per_wave, "bucket_order": t.bucket_order,
             "delta_d": t.delta_d, "ms": round(float(t.ms), 4)} for t in table]
    return sched, rows


@_on_stream
def pdx_exact_tune(index: PdxIndex, q: torch.Tensor, k: int, mode: str = "bond", metric: str = "l2",
                   chunk: int = 0, tile_groups: int = 0, queries_per_block: int = 0, reps: int = 3,
                   stream: Optional[torch.cuda.Stream] = None):
    """Fastest tile-scan schedule for this exact search (pdx_exact_tune).
    Returns (schedule, table): schedule = keyword arguments for
    pdx_search_exact (start_rows, rounds, dense_min); table = every
    candidate with its best time in ms (-1: skipped)."""
    q = _dev_f32(q, "q")
    nq = q.shape[0]
    if q.shape[1] != index.d:
        raise ValueError("query dimension does not match the index")
    p = _lib.pdx_search_params(_MODES[mode], chunk, tile_groups, queries_per_block, None, None, _METRICS[metric])
    need = lib.pdx_exact_tune_workspace(index.handle, nq, k, ctypes.byref(p))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=q.device)
    table = (_lib.pdx_exact_schedule * _lib.EXACT_TUNE_CANDIDATES)()
    _hold_index(index)
    st = lib.pdx_exact_tune(index.handle, _ptr(q), nq, k, ctypes.byref(p), int(reps), table, _ptr(ws), ws.numel(),
                            _stream(stream))
    check(st, "pdx_exact_tune")
    sched = {"start_rows": p.start_rows, "rounds": p.rounds, "dense_min": p.dense_min}
    rows = [{"start_rows": t.start_rows, "rounds": t.rounds, "dense_min": t.dense_min, "ms": round(float(t.ms), 4)}
            for t in table]
    return sched, rows


@_on_stream
def pdx_layout_blocks(x: torch.Tensor, block: int = 64,
                      stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """Rows [n, d] -> PDX blocks [ceil(n / block), d, block] (Section 3),
    the last block zero-padded."""
    x = _dev_f32(x, "x")
    n, d = x.shape
    nbytes = lib.pdx_layout_blocks_bytes(n, d, int(block))
    if nbytes == 0:
        raise ValueError("pdx_layout_blocks: need n, d >= 1 and block in 16, 32, 64, 128, 256, 512")
    out = torch.empty(((n + block - 1) // block, d, block), dtype=torch.float32, device=x.device)
    check(lib.pdx_layout_blocks(_ptr(x), n, d, int(block), _ptr(out), _stream(stream)), "pdx_layout_blocks")
    return out


@_on_stream
def pdx_distances(data: torch.Tensor, q: torch.Tensor, n: Optional[int] = None, layout: str = "pdx",
                  metric: str = "l2", stream: Optional[torch.cuda.Stream] = None,
                  out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Scores of every vector for each query, no search: [nq, n] float32.
    layout "nary": data = rows [n, d]; layout "pdx": data = the blocks of
    pdx_layout_blocks [nblocks, d, block] (block read from the shape) and n
    the number of real vectors (default: every slot)."""
    q = _dev_f32(q, "q")
    if not isinstance(data, torch.Tensor) or not data.is_cuda or data.dtype != torch.float32:
        raise TypeError("data must be a float32 GPU tensor")
    data = data.contiguous()
    if layout == "nary":
        if data.dim() != 2:
            raise TypeError("row-major data must be [n, d]")
        nn, d = data.shape
        block = 0
    elif layout == "pdx":
        if data.dim() != 3:
            raise TypeError("PDX data must be [nblocks, d, block]")
        nb, d, block = data.shape
        nn = nb * block if n is None else int(n)
        if not (nb - 1) * block < nn <= nb * block:
            raise ValueError("n does not match the number of blocks")
    else:
        raise ValueError(f"unknown layout {layout!r}")
    if q.shape[1] != d:
        raise ValueError("query dimension does not match the data")
    nq = q.shape[0]
    if out is None:
        out = torch.empty((nq, nn), dtype=torch.float32, device=q.device)
    elif out.dtype != torch.float32 or not out.is_contiguous() or out.numel() != nq * nn:
        raise TypeError("out must be contiguous float32 [nq, n]")
    lay = _lib.PDX_LAYOUT_NARY if layout == "nary" else _lib.PDX_LAYOUT_PDX
    check(lib.pdx_distances(_ptr(data), lay, int(block), nn, d, _ptr(q), nq, _METRICS[metric], _ptr(out),
                            _stream(stream)), "pdx_distances")
    return out


def pdx_version() -> str:
    return lib.pdx_version().decode()
