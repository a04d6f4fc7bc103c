"""MI355X-native evaluator for the cuROB test functions (arXiv 1407.7737).

Thin Python binding over libcurob.so with the names of the paper's interface (Sec. 1.3):
``initialize``, ``dispose``, ``func_evaluate`` (FP64), ``func_evaluatef`` (FP32), the host
wrappers ``h_func_evaluate`` / ``h_func_evaluatef``, plus the library extensions.  Torch
tensors provide device memory and the stream; all evaluation happens in the HIP kernels.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import _native
from ._native import (CUROB_E_ARG, CUROB_E_CAPACITY, CUROB_E_FID, CUROB_E_HIP, CUROB_E_STATE, CUROB_OK,
                      CUSTOM_ID_MAX, CUSTOM_ID_MIN, MODE_FP32, MODE_SPLIT, MODE_SPLIT_BF16X3,
                      MODE_SPLIT_BF16X6, CurobError, check, last_error)

lib = _native.lib

# Tab. 1 ids
SPHERE, ELLIPSOID, ELLIPTIC, DISCUS, CIGAR, POWERS, SHARPV = range(7)
STEP, WEIERSTRASS, GRIEWANK, RASTRIGIN_U, RASTRIGIN, SCHAFFERSF7 = range(7, 13)
GRIE_ROSEN, ROSENBROCK, SCHWEFEL_U, SCHWEFEL, KATSUURA, LUNACEK = range(13, 19)
ACKLEY, HAPPYCAT, HGBAT, SCHAFFERSF6 = range(19, 23)
HYBRID1, COMPOSITION1 = 23, 29

__all__ = [
    "initialize", "dispose", "func_evaluate", "func_evaluatef", "h_func_evaluate", "h_func_evaluatef",
    "set_stream", "set_mode", "define_basic", "define_hybrid", "define_composition", "get_problem",
    "generate_basic", "get_dim", "get_structure", "get_composition", "generate_structure",
    "generate_composition", "last_error", "CurobError", "Batch", "DE", "tune", "shape_key",
]

# dimension given to initialize, for the shape checks of the device calls (None: not initialised
# through this binding; the library is then asked)
_dim = None


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _torch_stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def initialize(dim: int, max_concurrency: int, seed: int = 0) -> None:
    global _dim
    check(lib.initialize(int(dim), int(max_concurrency), int(seed)))
    _dim = int(dim)


def dispose() -> None:
    global _dim
    _dim = None
    check(lib.dispose())


def get_dim() -> tuple:
    """(dim, max_concurrency) given to initialize."""
    d, m = ctypes.c_int(), ctypes.c_int()
    check(lib.curob_get_dim(ctypes.byref(d), ctypes.byref(m)))
    return d.value, m.value


def _current_dim() -> int:
    return _dim if _dim is not None else get_dim()[0]


def set_stream(stream=None) -> None:
    """Stream for device-pointer calls: a torch.cuda.Stream, a raw hipStream_t or None."""
    if stream is None:
        h = None
    elif isinstance(stream, int):
        h = stream
    else:
        h = stream.cuda_stream
    check(lib.curob_set_stream(h))


def set_mode(mode: int) -> None:
    check(lib.curob_set_mode(int(mode)))


def _eval_device(fn, fid, x, out, dtype_name):
    import torch
    want = torch.float64 if dtype_name == "f64" else torch.float32
    if not (x.is_cuda and x.dtype == want and x.is_contiguous() and x.dim() == 2):
        raise ValueError(f"x must be a contiguous 2-D {want} CUDA tensor")
    dim = _current_dim()
    if x.shape[1] != dim:
        raise ValueError(f"x has rows of {x.shape[1]} elements, the library was initialised with dim {dim}")
    n = x.shape[0]
    if out is None:
        out = torch.empty(n, dtype=want, device=x.device)
    elif not (out.is_cuda and out.dtype == want and out.is_contiguous() and out.numel() >= n):
        raise ValueError(f"out must be a contiguous {want} CUDA tensor with at least {n} entries")
    check(lib.curob_set_stream(_torch_stream()))
    check(fn(int(fid), _ptr(x), int(n), _ptr(out)))
    return out


def func_evaluate(fid: int, x, out=None):
    """FP64 evaluation of n x dim device rows; returns the (n,) device result."""
    return _eval_device(lib.func_evaluate, fid, x, out, "f64")


def func_evaluatef(fid: int, x, out=None):
    """FP32 evaluation (BF16 split rotation by default, see set_mode)."""
    return _eval_device(lib.func_evaluatef, fid, x, out, "f32")


def func_evaluate_ptr(fid: int, d_x: int, n: int, d_out: int) -> None:
    """Raw device-pointer form of func_evaluate (no checks beyond the library's own)."""
    check(lib.func_evaluate(int(fid), d_x, int(n), d_out))


def func_evaluatef_ptr(fid: int, d_x: int, n: int, d_out: int) -> None:
    check(lib.func_evaluatef(int(fid), d_x, int(n), d_out))


def _eval_host(fn, fid, x, dt):
    x = np.ascontiguousarray(np.asarray(x, dtype=dt))
    if x.ndim == 1:
        x = x[None, :]
    dim = _current_dim()
    if x.ndim != 2 or x.shape[1] != dim:
        raise ValueError(f"x must have rows of {dim} elements (got shape {x.shape})")
    out = np.empty(x.shape[0], dtype=dt)
    check(fn(int(fid), x.ctypes.data, int(x.shape[0]), out.ctypes.data))
    return out


def h_func_evaluate(fid: int, x) -> np.ndarray:
    """Host-pointer FP64 evaluation (copies in, evaluates, copies out, waits)."""
    return _eval_host(lib.h_func_evaluate, fid, x, np.float64)


def h_func_evaluatef(fid: int, x) -> np.ndarray:
    return _eval_host(lib.h_func_evaluatef, fid, x, np.float32)


def define_basic(pid: int, base: int, scale: float, offset: float = 0.0, rotated: bool = True) -> None:
    check(lib.curob_define_basic(int(pid), int(base), float(scale), float(offset), int(bool(rotated))))


def define_hybrid(pid: int, bases, p) -> None:
    b = np.ascontiguousarray(bases, dtype=np.int32)
    pp = np.ascontiguousarray(p, dtype=np.float64)
    check(lib.curob_define_hybrid(int(pid), len(b), b.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                  pp.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))


def define_composition(pid: int, bases, sigma, lam, bias) -> None:
    b = np.ascontiguousarray(bases, dtype=np.int32)
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (sigma, lam, bias)]
    dp = ctypes.POINTER(ctypes.c_double)
    check(lib.curob_define_composition(int(pid), len(b), b.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                       *[a.ctypes.data_as(dp) for a in arrs]))


def get_problem(fid: int, dim: int | None = None):
    """Shift o and dense rotation R of a basic problem of the initialised library.  `dim`, if
    given, must equal the initialised dimension (the buffers are sized from the library's)."""
    d = _current_dim()
    if dim is not None and int(dim) != d:
        raise ValueError(f"the library was initialised with dim {d}, not {dim}")
    dim = d
    o = np.empty(dim)
    R = np.empty((dim, dim))
    dp = ctypes.POINTER(ctypes.c_double)
    check(lib.curob_get_problem(int(fid), o.ctypes.data_as(dp), R.ctypes.data_as(dp)))
    return o, R


def generate_basic(fid: int, dim: int, seed: int):
    """Host-only: the shift and dense rotation initialize(dim, ..., seed) draws for fid."""
    o = np.empty(dim)
    R = np.empty((dim, dim))
    dp = ctypes.POINTER(ctypes.c_double)
    check(lib.curob_generate_basic(int(fid), int(dim), int(seed), o.ctypes.data_as(dp), R.ctypes.data_as(dp)))
    return o, R


def _structure(info_fn, struct_fn, lead, comp):
    """Unpacks the curob_*_info / curob_*_structure pair (see include/curob.h)."""
    t, cnt, ns = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    check(info_fn(*lead, int(comp), ctypes.byref(t), ctypes.byref(cnt), ctypes.byref(ns)))
    res = {"type": ("basic", "hybrid", "composition")[t.value], "count": cnt.value}
    if t.value == 2 and comp < 0:
        return res
    # sizes first (blocks need their total)
    sizes = np.zeros(max(cnt.value, 1), dtype=np.int32)
    dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    check(struct_fn(*lead, int(comp), None, None, sizes.ctypes.data_as(ip), None, None, None, None))
    sizes = sizes[:cnt.value]
    dim = lead[-2] if len(lead) == 3 else _current_dim()
    o = np.empty(dim)
    perm = np.empty(dim, dtype=np.int32)
    blocks = np.empty(max(int(np.sum(sizes.astype(np.int64) ** 2)), 1))
    bases = np.empty(max(ns.value, 1), dtype=np.int32)
    scale, offset = np.empty(max(ns.value, 1)), np.empty(max(ns.value, 1))
    check(struct_fn(*lead, int(comp), o.ctypes.data_as(dp), perm.ctypes.data_as(ip), sizes.ctypes.data_as(ip),
                    blocks.ctypes.data_as(dp), bases.ctypes.data_as(ip), scale.ctypes.data_as(dp),
                    offset.ctypes.data_as(dp)))
    mats, off = [], 0
    for n in sizes:
        mats.append(blocks[off:off + n * n].reshape(n, n).copy())
        off += n * n
    res.update(o=o, perm=perm, sizes=sizes, blocks=mats, bases=bases[:ns.value].copy(),
               scale=scale[:ns.value].copy(), offset=offset[:ns.value].copy())
    return res


def _blend(fn, lead):
    sig, lam, bias = np.zeros(16), np.zeros(16), np.zeros(16)
    dp = ctypes.POINTER(ctypes.c_double)
    check(fn(*lead, sig.ctypes.data_as(dp), lam.ctypes.data_as(dp), bias.ctypes.data_as(dp)))
    return sig, lam, bias


def get_structure(fid: int, comp: int = -1) -> dict:
    """Structure of problem fid (or of component comp of a composition) in the initialised
    library: type, count and, for basic and hybrid parts, o, perm (S), block sizes, blocks,
    and per formula segment its Tab. 1 id, scale and offset (curob_get_structure)."""
    return _structure(lib.curob_get_info, lib.curob_get_structure, (int(fid),), comp)


def generate_structure(fid: int, dim: int, seed: int, comp: int = -1) -> dict:
    """Host-only form of get_structure for Tab. 1 id fid at (dim, seed); no device needed."""
    return _structure(lib.curob_generate_info, lib.curob_generate_structure, (int(fid), int(dim), int(seed)), comp)


def get_composition(fid: int):
    """(sigma, lambda, bias) of a composition of the initialised library."""
    n = get_structure(fid)["count"]
    return tuple(a[:n] for a in _blend(lib.curob_get_composition, (int(fid),)))


def generate_composition(fid: int, dim: int, seed: int):
    """Host-only (sigma, lambda, bias) of Tab. 1 composition fid at (dim, seed)."""
    n = generate_structure(fid, dim, seed)["count"]
    return tuple(a[:n] for a in _blend(lib.curob_generate_composition, (int(fid), int(dim), int(seed))))


def probe_read_gbs(x, reps: int = 10) -> float:
    """Measured streaming read bandwidth (GB/s) over the device tensor x (curob_probe_read)."""
    gbs = ctypes.c_double()
    check(lib.curob_probe_read(_ptr(x), int(x.numel() * x.element_size()), int(reps), ctypes.byref(gbs)))
    return gbs.value


def probe_mfma_bf16_tflops(reps: int = 5) -> float:
    """Measured dense BF16 16x16x32 MFMA rate (TFLOP/s) (curob_probe_mfma_bf16)."""
    tf = ctypes.c_double()
    check(lib.curob_probe_mfma_bf16(int(reps), ctypes.byref(tf)))
    return tf.value


def _arch() -> str:
    import torch
    prop = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{getattr(prop, 'gcnArchName', 'gpu')}|{prop.name}|{prop.multi_processor_count}cu"


def shape_key(fid: int, n: int, fp64: bool = False) -> str:
    """Cache key of the launch shape of fid on n rows: architecture, path, D bucket, formula
    class and row bucket (curob_shape_key)."""
    k = (ctypes.c_int * 4)()
    check(lib.curob_shape_key(int(fid), int(bool(fp64)), int(n), k))
    return f"{_arch()}|path{k[0]}|d{k[1]}|class{k[2]}|n{k[3]}"


def tune(fid: int, x, fp64: bool = False, reps: int = 10, cache: str | None = None) -> dict:
    """Autotunes the single-call launch shape of fid for x's row count (curob_tune) on x and a
    scratch output, or applies the entry of the JSON cache for the same key.  Returns the chosen
    shape with its time and, when freshly tuned, the search log (one entry per candidate)."""
    import json

    import torch
    key = shape_key(fid, x.shape[0], fp64)
    k4 = (ctypes.c_int * 4)()
    check(lib.curob_shape_key(int(fid), int(bool(fp64)), int(x.shape[0]), k4))
    entries = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            entries = json.load(f)
        if key in entries:
            e = entries[key]
            check(lib.curob_set_shape(k4, int(e["waves"]), int(e["grid_per8"])))
            return dict(e, key=key, cached=True)
    want = torch.float64 if fp64 else torch.float32
    if not (x.is_cuda and x.dtype == want and x.is_contiguous() and x.dim() == 2 and x.shape[1] == _current_dim()):
        raise ValueError(f"x must be a contiguous (n, dim) {want} CUDA tensor")
    out = torch.empty(x.shape[0], dtype=want, device=x.device)
    bw, bg = ctypes.c_int(), ctypes.c_int()
    bus = ctypes.c_float()
    cap = 64
    log = (ctypes.c_float * (3 * cap))()
    nlog = ctypes.c_int()
    check(lib.curob_set_stream(_torch_stream()))
    check(lib.curob_tune(int(fid), int(bool(fp64)), _ptr(x), int(x.shape[0]), _ptr(out), int(reps), ctypes.byref(bw),
                         ctypes.byref(bg), ctypes.byref(bus), log, cap, ctypes.byref(nlog)))
    res = {"waves": bw.value, "grid_per8": bg.value, "us": round(float(bus.value), 3)}
    if cache:
        entries[key] = res
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(entries, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    search = [{"waves": int(log[3 * i]), "grid_per8": int(log[3 * i + 1]), "us": round(float(log[3 * i + 2]), 3)}
              for i in range(nlog.value)]
    return dict(res, key=key, cached=False, search=search)


class DE:
    """Differential evolution (DE/rand/1/bin) on the GPU around func_evaluate[f]
    (curob_de_run): population, values, work space and the generation counter are device
    tensors owned here.  run(k) enqueues k generations on torch's current stream; capture(k)
    records k generations in one CUDA/HIP graph that replay() runs again (continuing from the
    device generation counter)."""

    def __init__(self, fid: int, pop, F: float = 0.5, CR: float = 0.9, seed: int = 0, fp64: bool = True):
        import torch
        want = torch.float64 if fp64 else torch.float32
        if not (pop.is_cuda and pop.dtype == want and pop.is_contiguous() and pop.dim() == 2):
            raise ValueError(f"pop must be a contiguous 2-D {want} CUDA tensor")
        if pop.shape[1] != _current_dim():
            raise ValueError("population rows must have the initialised dimension")
        self.fid, self.F, self.CR, self.seed, self.fp64 = int(fid), float(F), float(CR), int(seed), bool(fp64)
        self.pop = pop.clone()
        self.np = int(pop.shape[0])
        self.trial = torch.empty_like(self.pop)
        self.ftrial = torch.empty(self.np, dtype=want, device=pop.device)
        self.gen = torch.zeros(1, dtype=torch.int64, device=pop.device)
        self.fit = (func_evaluate if fp64 else func_evaluatef)(self.fid, self.pop).clone()
        self.graph = None

    def run(self, generations: int) -> None:
        check(lib.curob_set_stream(_torch_stream()))
        check(lib.curob_de_run(self.fid, int(self.fp64), self.np, self.F, self.CR, self.seed, _ptr(self.pop),
                               _ptr(self.fit), _ptr(self.trial), _ptr(self.ftrial), _ptr(self.gen), int(generations)))

    def capture(self, generations: int) -> None:
        """Records `generations` generations (trials, evaluation, selection) in one graph."""
        import torch
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                self.run(generations)
        torch.cuda.current_stream().wait_stream(s)
        check(lib.curob_set_stream(_torch_stream()))
        self.graph = g

    def replay(self) -> None:
        self.graph.replay()


class Batch:
    """Populations of uneven size, dimension and function evaluated by one persistent launch
    replayed as a HIP graph (curob_batch_*).  Population i is Tab. 1 function fids[i] at
    dimension dims[i] with counts[i] rows, its random data keyed like custom id 2048 + i."""

    def __init__(self, fids, dims, counts, seed: int = 0):
        self.k = len(fids)
        arr = [np.ascontiguousarray(a, dtype=np.int32) for a in (fids, dims, counts)]
        ip = ctypes.POINTER(ctypes.c_int)
        h = ctypes.c_void_p()
        check(lib.curob_batch_create(self.k, *[a.ctypes.data_as(ip) for a in arr], int(seed), ctypes.byref(h)))
        self._h = h
        self.fids, self.dims, self.counts = (a.copy() for a in arr)
        self.seed = int(seed)

    def bind(self, xs, outs) -> None:
        """xs[i]: (counts[i], dims[i]) float32 CUDA tensor; outs[i]: (counts[i],) float32."""
        import torch
        if len(xs) != self.k or len(outs) != self.k:
            raise ValueError("one input and one output buffer per population")
        for i, (x, o) in enumerate(zip(xs, outs)):
            if self.counts[i] == 0:
                continue
            if x.dtype != torch.float32 or o.dtype != torch.float32 or not x.is_cuda or not o.is_cuda:
                raise TypeError("batch buffers are float32 CUDA tensors")
            if tuple(x.shape) != (int(self.counts[i]), int(self.dims[i])) or not x.is_contiguous():
                raise ValueError(f"population {i}: expected a contiguous ({self.counts[i]}, {self.dims[i]}) input")
            if o.numel() < self.counts[i] or not o.is_contiguous():
                raise ValueError(f"population {i}: output needs {self.counts[i]} contiguous entries")
        X = (ctypes.c_void_p * self.k)(*[_ptr(t) if t is not None and t.numel() else None for t in xs])
        O = (ctypes.c_void_p * self.k)(*[_ptr(t) if t is not None and t.numel() else None for t in outs])
        self._keep = (xs, outs)
        check(lib.curob_set_stream(_torch_stream()))
        check(lib.curob_batch_bind(self._h, X, O))

    def run(self) -> None:
        """Replays the captured graph on torch's current stream."""
        check(lib.curob_set_stream(_torch_stream()))
        check(lib.curob_batch_run(self._h))

    def run_direct(self) -> None:
        """The same persistent launch without the graph."""
        check(lib.curob_set_stream(_torch_stream()))
        check(lib.curob_batch_run_direct(self._h))

    def configure(self, waves: int, groups_per_item: int, grid: int) -> None:
        check(lib.curob_batch_configure(self._h, int(waves), int(groups_per_item), int(grid)))

    def shape(self) -> dict:
        v = [ctypes.c_int() for _ in range(4)]
        check(lib.curob_batch_shape(self._h, *[ctypes.byref(a) for a in v]))
        return dict(zip(("waves", "groups_per_item", "grid", "items"), (a.value for a in v)))

    def signature(self) -> str:
        """Tuning-cache key: architecture, path (the split path), the largest dimension's bucket
        (<= 16, 32, 64, 96, 128), and log2 buckets of the total row count and of the number of
        populations -- batches alike in these share a launch shape."""
        dmax = int(self.dims.max()) if self.k else 0
        dbucket = 0 if dmax <= 16 else 1 if dmax <= 32 else 2 if dmax <= 64 else 3 if dmax <= 96 else 4
        rows = max(1, int(self.counts.sum()))
        return f"{_arch()}|batch-split|d{dbucket}|rows{rows.bit_length() - 1}|pops{max(1, self.k).bit_length() - 1}"

    def tune(self, reps: int = 20, cache: str | None = None) -> dict:
        """Autotunes the launch shape on the bound buffers (curob_batch_tune).  With a cache
        path (JSON), a shape stored under the same key (signature()) is applied without timing,
        and a freshly tuned one is stored."""
        import json
        key = self.signature()
        entries = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                entries = json.load(f)
            if key in entries:
                e = entries[key]
                self.configure(e["waves"], e["groups_per_item"], e["grid"])
                return dict(self.shape(), us=e.get("us"), cached=True)
        check(lib.curob_set_stream(_torch_stream()))
        best = ctypes.c_float()
        check(lib.curob_batch_tune(self._h, int(reps), ctypes.byref(best)))
        res = dict(self.shape(), us=float(best.value), cached=False)
        if cache:
            entries[key] = {k: res[k] for k in ("waves", "groups_per_item", "grid", "us")}
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(entries, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return res

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib.curob_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
