"""Torch-facing wrapper over the C-ABI (device memory and streams only).

All computation happens in the HIP library; this module only turns torch
device tensors into pointers and sizes, and the current torch stream into the
``hipStream_t`` handle.
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np

from . import capi as C


def _torch():
    import torch
    return torch


def _stream_handle(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(0)


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return C.SPMV_F64
    if t.dtype == torch.float32:
        return C.SPMV_F32
    raise TypeError(f"values must be float32 or float64, got {t.dtype}")


def make_csr(row_ptr, col, val, n):
    """spmv_csr view of torch device tensors (int32 row_ptr/col, f32/f64 val)."""
    torch = _torch()
    for name, t, dt in (("row_ptr", row_ptr, torch.int32), ("col", col, torch.int32)):
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous int32 device tensor")
    if not val.is_cuda or not val.is_contiguous():
        raise TypeError("val must be a contiguous device tensor")
    m = row_ptr.numel() - 1
    return C.spmv_csr(m, int(n), int(col.numel()), _ptr(row_ptr), _ptr(col), _ptr(val),
                      _dtype_code(val))


def _struct_to_dict(s):
    out = {}
    for name, _ in s._fields_:
        v = getattr(s, name)
        if isinstance(v, ctypes.Structure):
            v = _struct_to_dict(v)
        elif isinstance(v, ctypes.Array):
            v = list(v)
        out[name] = v
    return out


def features(row_ptr, col, val, n, stream=None):
    """GPU feature extraction (validation included) as a dict."""
    A = make_csr(row_ptr, col, val, n)
    F = C.spmv_features()
    C.check(C.lib().spmv_features_compute(ctypes.byref(A), ctypes.byref(F), _stream_handle(stream)),
            "spmv_features_compute")
    return _struct_to_dict(F)


class Selector:
    """Learned selector weights uploaded to the device."""

    def __init__(self, params, mean, std):
        p = np.ascontiguousarray(params, dtype=np.float32)
        mu = np.ascontiguousarray(mean, dtype=np.float32)
        sd = np.ascontiguousarray(std, dtype=np.float32)
        h = ctypes.c_void_p()
        C.check(C.lib().spmv_selector_create(p.ctypes.data_as(ctypes.c_void_p), p.size,
                                             mu.ctypes.data_as(ctypes.c_void_p),
                                             sd.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)),
                "spmv_selector_create")
        self.handle = h
        self.params, self.mean, self.std = p, mu, sd
        self.lo = self.hi = None
        self.stage = None

    @classmethod
    def load(cls, path):
        with open(path) as fh:
            d = json.load(fh)
        sel = cls(d["params"], d["mean"], d["std"])
        sel.tau = d.get("meta", {}).get("tau")
        if "lo" in d and "hi" in d:
            sel.set_domain(d["lo"], d["hi"])
        if "stage" in d:
            sel.set_stage(d["stage"])
        return sel

    def set_stage(self, rule):
        """Stage rule for staged plans: a dict of equal-length node lists
        feat, thr, left, right, kernel, conf (see spmv_selector_set_stage);
        None removes it."""
        if rule is None:
            C.check(C.lib().spmv_selector_set_stage(self.handle, None, None, None, None, None,
                                                    None, 0), "spmv_selector_set_stage")
            self.stage = None
            return
        arr = {k: np.ascontiguousarray(rule[k], dtype=np.float32 if k in ("thr", "conf")
                                       else np.int32)
               for k in ("feat", "thr", "left", "right", "kernel", "conf")}
        n = len(arr["feat"])
        assert all(len(v) == n for v in arr.values())
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        C.check(C.lib().spmv_selector_set_stage(self.handle, ptr(arr["feat"]), ptr(arr["thr"]),
                                                ptr(arr["left"]), ptr(arr["right"]),
                                                ptr(arr["kernel"]), ptr(arr["conf"]), n),
                "spmv_selector_set_stage")
        self.stage = arr

    def set_domain(self, lo, hi):
        """Training range of the 12 raw inputs (None, None clears it)."""
        if lo is None and hi is None:
            C.check(C.lib().spmv_selector_set_domain(self.handle, None, None),
                    "spmv_selector_set_domain")
            self.lo = self.hi = None
            return
        lo = np.ascontiguousarray(lo, dtype=np.float32)
        hi = np.ascontiguousarray(hi, dtype=np.float32)
        assert lo.shape == (12,) and hi.shape == (12,)
        C.check(C.lib().spmv_selector_set_domain(self.handle, lo.ctypes.data_as(ctypes.c_void_p),
                                                 hi.ctypes.data_as(ctypes.c_void_p)),
                "spmv_selector_set_domain")
        self.lo, self.hi = lo, hi

    def score(self, raw, stream=None):
        """raw: float32 device tensor [rows, 12] -> scores [rows, K_COUNT]."""
        torch = _torch()
        raw = raw.to(torch.float32).contiguous()
        out = torch.empty((raw.shape[0], C.K_COUNT), dtype=torch.float32, device=raw.device)
        C.check(C.lib().spmv_selector_score(self.handle, _ptr(raw), raw.shape[0], _ptr(out),
                                            _stream_handle(stream)), "spmv_selector_score")
        return out

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and C._lib is not None:
            C.lib().spmv_selector_destroy(h)
            self.handle = None


DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                               "selector_gfx950.json")


def weights_path():
    """The selector weights file: $SPMV_WEIGHTS when set (non-empty), else the
    shipped one."""
    return os.environ.get("SPMV_WEIGHTS") or DEFAULT_WEIGHTS


def default_selector():
    """The trained selector of weights_path(), or None if the file is absent
    or was trained for another kernel set."""
    path = weights_path()
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        meta = json.load(fh)
    if meta.get("n_out") != C.K_COUNT or list(meta.get("kernels", [])) != list(C.KERNELS):
        return None
    return Selector.load(path)


class TorchAllocator:
    """Plan memory from PyTorch's caching allocator (spmv_allocator): every
    block is a uint8 tensor on the device, held until the library frees it.

    Blocks are allocated for the stream the plan is created on (``stream``,
    set by Plan while it creates), so a block the library frees during plan
    creation is only reused by PyTorch after the work already queued on that
    stream; spmv_plan_destroy synchronises the device before it frees the
    plan's own blocks, so runs on any stream have ended by then."""

    def __init__(self, device):
        self.device = device
        self.blocks = {}
        self.stream = None

        def alloc(nbytes, ctx):
            torch = _torch()
            try:
                if self.stream is not None:
                    with torch.cuda.stream(self.stream):
                        t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
                else:
                    t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            except Exception:  # out of memory: the library reports ENOMEM
                return None
            self.blocks[t.data_ptr()] = t
            return t.data_ptr()

        def free(ptr, nbytes, ctx):
            try:
                self.blocks.pop(ptr, None)
            except Exception:  # interpreter shutting down
                pass

        self._alloc = C.ALLOC_FN(alloc)   # the callbacks must outlive every plan
        self._free = C.FREE_FN(free)

    def fill(self, opts):
        opts.allocator.alloc = self._alloc
        opts.allocator.free = self._free
        opts.allocator.ctx = None

    def bytes_held(self):
        return sum(t.numel() for t in self.blocks.values())


_TORCH_ALLOCATORS = {}


def torch_allocator(device):
    """The process-wide TorchAllocator of a device."""
    torch = _torch()
    device = torch.device(device)
    if device.index is None:
        device = torch.device(device.type, torch.cuda.current_device())
    if device not in _TORCH_ALLOCATORS:
        _TORCH_ALLOCATORS[device] = TorchAllocator(device)
    return _TORCH_ALLOCATORS[device]


class Plan:
    """spmv_plan_create / spmv_run over torch device tensors.

    selector: "rules", "mlp", "exhaustive", or a kernel name / index to force.
    """

    def __init__(self, row_ptr, col, val, n=None, selector="rules", model=None,
                 tau=None, topk=None, reps=None, disable=(), mem_cap=0, params=None,
                 autotune=False, segments=0, staged=True, stage_conf=None,
                 allocator="torch", stream=None, time_baseline=False, log=False):
        torch = _torch()
        m = row_ptr.numel() - 1
        n = m if n is None else int(n)
        A = make_csr(row_ptr, col, val, n)
        o = C.spmv_plan_opts()
        C.lib().spmv_plan_opts_default(ctypes.byref(o))
        if isinstance(selector, int) or selector in C.KERNELS:
            o.selector = C.SELECT_FORCED
            o.force_kernel = selector if isinstance(selector, int) else C.KERNELS.index(selector)
        else:
            o.selector = {"rules": C.SELECT_RULES, "mlp": C.SELECT_MLP,
                          "exhaustive": C.SELECT_EXHAUSTIVE}[selector]
        if selector == "mlp":
            model = model or default_selector()
            if model is None:
                raise RuntimeError("selector='mlp' needs a model (no trained weights found)")
        self._model = model
        o.model = model.handle if model is not None else None
        if tau is not None:
            o.confidence_tau = tau
        if topk is not None:
            o.measure_topk = topk
        if reps is not None:
            o.timing_reps = reps
        mask = 0
        for k in disable:
            mask |= 1 << (k if isinstance(k, int) else C.KERNELS.index(k))
        o.disable_mask = mask
        o.mem_cap_bytes = int(mem_cap)
        o.autotune = 1 if autotune else 0
        o.time_baseline = 1 if time_baseline else 0
        o.log = 1 if log else 0
        o.segments = int(segments)
        o.staged = 1 if staged else 0
        if stage_conf is not None:
            o.stage_conf = float(stage_conf)
        # plan memory from torch's caching allocator ("torch"), the library's
        # hipMalloc (None), or a TorchAllocator given by the caller
        self._allocator = torch_allocator(val.device) if allocator == "torch" else allocator
        if self._allocator is not None:
            self._allocator.fill(o)
        if selector == "mlp" and tau is None and model is not None and \
                getattr(model, "tau", None) is not None:
            o.confidence_tau = model.tau
        if params:
            o.use_params = 1
            for k, v in params.items():
                setattr(o.params, k, int(v))
        h = ctypes.c_void_p()
        if val.device.type != "cuda" or row_ptr.device != val.device or col.device != val.device:
            raise TypeError("row_ptr, col and val must be tensors on one GPU")
        with torch.cuda.device(val.device):   # the library works on the current device
            cs = stream if stream is not None else torch.cuda.current_stream()
            if self._allocator is not None:
                self._allocator.stream = cs
            try:
                st = C.lib().spmv_plan_create(ctypes.byref(A), ctypes.byref(o),
                                              _stream_handle(cs), ctypes.byref(h))
            finally:
                if self._allocator is not None:
                    self._allocator.stream = None
        C.check(st, "spmv_plan_create")
        self.handle = h
        self.m, self.n, self.nnz = m, n, int(col.numel())
        self.dtype = val.dtype
        self.device = val.device

    def run(self, x, y=None, stream=None, out=None):
        """y = A x on the current torch stream (or `stream`); y (or `out`)
        is overwritten, or allocated when neither is given."""
        torch = _torch()
        if out is not None:
            if y is not None:
                raise TypeError("give y or out, not both")
            y = out
        if x.dtype != self.dtype or not x.is_contiguous() or x.numel() != self.n:
            raise TypeError("x must be a contiguous vector of length n and the matrix dtype")
        if y is None:
            y = torch.empty(self.m, dtype=self.dtype, device=self.device)
        elif y.dtype != self.dtype or not y.is_contiguous() or y.numel() != self.m:
            raise TypeError("y must be a contiguous vector of length m and the matrix dtype")
        if x.device != self.device or y.device != self.device:
            raise TypeError("x and y must be on the plan's device")
        if torch.cuda.current_device() == self.device.index:
            C.check(C.lib().spmv_run(self.handle, _ptr(x), _ptr(y), _stream_handle(stream)),
                    "spmv_run")
        else:
            with torch.cuda.device(self.device):   # the library works on the current device
                C.check(C.lib().spmv_run(self.handle, _ptr(x), _ptr(y), _stream_handle(stream)),
                        "spmv_run")
        return y

    __call__ = run

    def info(self):
        I = C.spmv_plan_info()
        C.check(C.lib().spmv_plan_info_get(self.handle, ctypes.byref(I)), "spmv_plan_info_get")
        d = _struct_to_dict(I)
        if d["n_segments"] > 0:
            d["kernel_name"] = d["format_name"] = "segmented"
        else:
            d["kernel_name"] = C.KERNELS[d["kernel"]]
            d["format_name"] = C.FORMATS[d["format"]]
        d["rules_kernel_name"] = C.KERNELS[d["rules_kernel"]] if d["rules_kernel"] >= 0 else None
        return d

    def segments(self):
        """[(row0, plan of that row segment)] of a segmented plan; the segment
        plans belong to this one (they are never destroyed on their own)."""
        out = []
        for k in range(self.info()["n_segments"]):
            h = ctypes.c_void_p()
            r0 = ctypes.c_int64(0)
            C.check(C.lib().spmv_plan_segment(self.handle, k, ctypes.byref(h), ctypes.byref(r0)),
                    "spmv_plan_segment")
            seg = _SegmentPlan(h, self)
            out.append((r0.value, seg))
        return out

    def roundtrip(self, stream=None):
        torch = _torch()
        rp = torch.empty(self.m + 1, dtype=torch.int32, device=self.device)
        col = torch.empty(max(1, self.nnz), dtype=torch.int32, device=self.device)
        val = torch.empty(max(1, self.nnz), dtype=self.dtype, device=self.device)
        C.check(C.lib().spmv_convert_roundtrip(self.handle, _ptr(rp), ctypes.c_void_p(col.data_ptr()),
                                               ctypes.c_void_p(val.data_ptr()),
                                               _stream_handle(stream)), "spmv_convert_roundtrip")
        return rp, col[:self.nnz], val[:self.nnz]

    def export(self, which, stream=None):
        """Internal array `which` (see spmv_plan_export) as a uint8 device tensor."""
        torch = _torch()
        n = ctypes.c_size_t(0)
        C.check(C.lib().spmv_plan_export(self.handle, which, None, 0, ctypes.byref(n),
                                         _stream_handle(stream)), "spmv_plan_export(size)")
        buf = torch.empty(max(1, n.value), dtype=torch.uint8, device=self.device)
        C.check(C.lib().spmv_plan_export(self.handle, which, ctypes.c_void_p(buf.data_ptr()),
                                         buf.numel(), None, _stream_handle(stream)),
                "spmv_plan_export")
        return buf[:n.value]

    def close(self):
        h = getattr(self, "handle", None)
        if h and C._lib is not None:
            C.lib().spmv_plan_destroy(h)
        self.handle = None

    def __del__(self):
        self.close()


class _SegmentPlan(Plan):
    """A row segment's plan inside a segmented plan (not owned)."""

    def __init__(self, handle, parent):  # noqa: D107 -- no plan creation here
        self.handle = handle
        self._parent = parent
        I = C.spmv_plan_info()
        C.check(C.lib().spmv_plan_info_get(handle, ctypes.byref(I)), "spmv_plan_info_get")
        self.m, self.n, self.nnz = int(I.m), int(I.n), int(I.nnz)
        self.dtype, self.device = parent.dtype, parent.device

    def close(self):
        self.handle = None


class TuneCache:
    """Chosen kernel and parameters per matrix structure, kept as JSON (the
    result of the paper's kernel search, reused instead of searched again).

    The key is the device architecture, the value type and the integer
    structure features (sizes, row-length moments, diagonals, bandwidth,
    4x4 blocks); matrices alike in all of them share an entry.  A hit plans
    with the recorded kernel and parameters (no selection, no search); a
    miss plans with selection and autotuning and records the outcome.
    Every kernel computes the same product, so a shared entry only affects
    speed.
    """

    KEY_FEATURES = ("m", "n", "nnz", "sum_rd", "sum_rd2", "max_rd", "min_rd", "ndiags",
                    "ntdiags", "bandwidth", "blocks4")

    def __init__(self, path=None):
        path = path or os.environ.get("SPMV_AUTOTUNE_CACHE")
        if not path:
            raise ValueError("TuneCache needs a path (or $SPMV_AUTOTUNE_CACHE)")
        self.path = path
        self.entries = {}
        if os.path.exists(path):
            with open(path) as fh:
                self.entries = json.load(fh)
        self.hits = self.misses = 0

    def key(self, row_ptr, col, val, n):
        torch = _torch()
        f = features(row_ptr, col, val, n)
        arch = torch.cuda.get_device_properties(val.device).gcnArchName.split(":")[0]
        dt = "float64" if val.dtype == torch.float64 else "float32"
        return "|".join([arch, dt] + [str(int(f[k])) for k in self.KEY_FEATURES])

    def plan(self, row_ptr, col, val, n=None, **kw):
        """A Plan from the cache, or a tuned one recorded into it."""
        n = row_ptr.numel() - 1 if n is None else int(n)
        k = self.key(row_ptr, col, val, n)
        e = self.entries.get(k)
        if e is not None:
            self.hits += 1
            return Plan(row_ptr, col, val, n=n, selector=e["kernel"], params=e["params"],
                        stream=kw.get("stream"))
        self.misses += 1
        kw.setdefault("autotune", True)
        p = Plan(row_ptr, col, val, n=n, **kw)
        info = p.info()
        if info["n_segments"] == 0:
            self.entries[k] = {"kernel": info["kernel_name"], "params": info["params"]}
        return p

    def save(self):
        tmp = self.path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(self.entries, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


class Batch:
    """spmv_batch_*: all levels in one persistent launch (mode 0) or a graph (1)."""

    def __init__(self, plans, mode=0):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        h = ctypes.c_void_p()
        C.check(C.lib().spmv_batch_create(arr, len(self.plans), int(mode), ctypes.byref(h)),
                "spmv_batch_create")
        self.handle = h
        self.mode = mode

    def run(self, xs, ys, stream=None):
        n = len(self.plans)
        xa = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        ya = (ctypes.c_void_p * n)(*[y.data_ptr() for y in ys])
        C.check(C.lib().spmv_batch_run(self.handle, xa, ya, _stream_handle(stream)),
                "spmv_batch_run")
        return ys

    def tune(self, xs, ys, reps=5, stream=None):
        """Pick the persistent grid size by timing; returns the grid."""
        n = len(self.plans)
        xa = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        ya = (ctypes.c_void_p * n)(*[y.data_ptr() for y in ys])
        g = ctypes.c_int32(0)
        C.check(C.lib().spmv_batch_tune(self.handle, xa, ya, int(reps), _stream_handle(stream),
                                        ctypes.byref(g)), "spmv_batch_tune")
        return g.value

    def shape(self):
        """(persistent grid, leading levels launched on their own)."""
        g, k = ctypes.c_int32(0), ctypes.c_int32(0)
        C.check(C.lib().spmv_batch_shape(self.handle, ctypes.byref(g), ctypes.byref(k)),
                "spmv_batch_shape")
        return g.value, k.value

    def close(self):
        h = getattr(self, "handle", None)
        if h and C._lib is not None:
            C.lib().spmv_batch_destroy(h)
        self.handle = None

    def __del__(self):
        self.close()


def stream_read(src, out=None, stream=None):
    """spmv_stream_read over a device tensor (16-byte multiple); returns the
    per-thread word sums (uint8 tensor of spmv_stream_read_out_bytes())."""
    torch = _torch()
    nbytes = src.numel() * src.element_size()
    if out is None:
        out = torch.empty(int(C.lib().spmv_stream_read_out_bytes()), dtype=torch.uint8,
                          device=src.device)
    C.check(C.lib().spmv_stream_read(_ptr(src), nbytes, _ptr(out), _stream_handle(stream)),
            "spmv_stream_read")
    return out


def stream_copy(dst, src, stream=None):
    nbytes = src.numel() * src.element_size()
    C.check(C.lib().spmv_stream_copy(_ptr(dst), _ptr(src), nbytes, _stream_handle(stream)),
            "spmv_stream_copy")
    return dst


def gather_probe(table, idx, val, out=None, stream=None):
    """spmv_gather_probe over device tensors (table and val of one float
    dtype, idx int32); returns the per-thread sums."""
    torch = _torch()
    if table.dtype != val.dtype or table.dtype not in (torch.float32, torch.float64) or \
            idx.dtype != torch.int32 or idx.numel() != val.numel():
        raise TypeError("table / val float32 or float64 alike, idx int32 of val's length")
    n = int(C.lib().spmv_gather_probe_threads())
    if out is None:
        out = torch.empty(n, dtype=table.dtype, device=table.device)
    assert out.numel() == n and out.dtype == table.dtype
    C.check(C.lib().spmv_gather_probe(_ptr(table), table.numel(), _ptr(idx), _ptr(val),
                                      idx.numel(), table.element_size(), _ptr(out),
                                      _stream_handle(stream)), "spmv_gather_probe")
    return out


# ---- selector training kernels -------------------------------------------------

def mlp_param_count(n_out=C.K_COUNT):
    return int(C.lib().spmv_mlp_param_count(n_out))


def mlp_forward(params, x, n_out=C.K_COUNT, stream=None):
    torch = _torch()
    B = x.shape[0]
    ws = torch.empty(int(C.lib().spmv_mlp_workspace_floats(B)), dtype=torch.float32, device=x.device)
    out = torch.empty((B, n_out), dtype=torch.float32, device=x.device)
    C.check(C.lib().spmv_mlp_forward(_ptr(params), n_out, _ptr(x), B, _ptr(out), _ptr(ws),
                                     _stream_handle(stream)), "spmv_mlp_forward")
    return out


def mlp_backward(params, x, target, mask, n_out=C.K_COUNT, grad=None, ws=None, loss=None,
                 stream=None):
    torch = _torch()
    B = x.shape[0]
    if ws is None:
        ws = torch.empty(int(C.lib().spmv_mlp_workspace_floats(B)), dtype=torch.float32,
                         device=x.device)
    if grad is None:
        grad = torch.empty_like(params)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
    C.check(C.lib().spmv_mlp_backward(_ptr(params), n_out, _ptr(x), _ptr(target), _ptr(mask), B,
                                      _ptr(grad), _ptr(loss), _ptr(ws), _stream_handle(stream)),
            "spmv_mlp_backward")
    return grad, loss


def mlp_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    C.check(C.lib().spmv_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), params.numel(),
                                  int(step), lr, beta1, beta2, eps, _stream_handle(stream)),
            "spmv_mlp_adam")
