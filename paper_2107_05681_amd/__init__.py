"""Python binding of libmeld.so, the MI355X melded-kernel library.

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch supplies device memory (``data_ptr()``) and the current stream.

The library must be built in-tree first (``__graft_entry__.build()`` or
``python paper_2107_05681_amd/build.py``); importing the functions below
without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmeld.so")

DIVERGENT = 0
MELDED = 1
AUTO = 2
MELDED_INPLACE = 3
_VARIANTS = {"divergent": DIVERGENT, "melded": MELDED, "auto": AUTO,
             "melded_inplace": MELDED_INPLACE,
             DIVERGENT: DIVERGENT, MELDED: MELDED, AUTO: AUTO, MELDED_INPLACE: MELDED_INPLACE}

OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED = 0, 1, 2, 3, 4
_STATUS = {1: "EINVAL", 2: "ENOMEM", 3: "EHIP", 4: "EUNSUPPORTED"}

# Every function the C header declares.
EXPORTS = ("meld_version", "meld_create", "meld_destroy", "meld_last_error", "meld_sort_u32",
           "meld_sort_u32_steps", "meld_segmented_sort_u32", "meld_segmented_sort_u32_staged",
           "meld_segmented_sort_check", "meld_set_option", "meld_probe_region",
           "meld_probe_network", "meld_probe_segments", "meld_tune", "meld_plan_describe",
           "meld_tune_choose", "meld_server_create", "meld_server_create_simulated",
           "meld_server_submit", "meld_server_poll", "meld_server_release", "meld_server_read",
           "meld_server_drain", "meld_server_stats_get", "meld_server_last_error",
           "meld_server_destroy",
           "meld_divergent_region_f32", "meld_region3_f32", "meld_region_lanetrips_f32",
           "meld_oddeven_sort_buckets_u32", "meld_merge_sort_u32", "meld_sort_plan_describe",
           "meld_sort_u32_timed", "meld_sort_u32_noalloc", "meld_probe_region_gathers",
           "meld_server_now")


class MeldError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class Side(ctypes.Structure):
    _fields_ = [("a", ctypes.c_float), ("off", ctypes.c_uint32),
                ("step", ctypes.c_uint32), ("trips", ctypes.c_uint32)]


class SideRange(ctypes.Structure):
    _fields_ = [("a", ctypes.c_float), ("off", ctypes.c_uint32), ("step", ctypes.c_uint32),
                ("trips_lo", ctypes.c_uint32), ("trips_hi", ctypes.c_uint32)]


_lib = None
_lock = threading.Lock()
# One library context per (device, stream): a context's scratch (sort tail,
# segmented-sort queues, merge and tuning buffers) is shared by every call on
# it, so calls on streams that may run concurrently must not share one.
_ctxs: dict[tuple[int, int], ctypes.c_void_p] = {}
_options: dict[int, dict[int, int]] = {}  # device -> option -> value, for every context


def load_library():
    """Loads libmeld.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build the HIP extension first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz, u64, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_int64
    st = ctypes.c_int
    lib.meld_version.restype = ctypes.c_int
    lib.meld_version.argtypes = []
    lib.meld_create.restype = st
    lib.meld_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
    lib.meld_destroy.restype = None
    lib.meld_destroy.argtypes = [vp]
    lib.meld_last_error.restype = ctypes.c_char_p
    lib.meld_last_error.argtypes = []
    lib.meld_sort_u32.restype = st
    lib.meld_sort_u32.argtypes = [vp, vp, vp, sz, st, vp]
    lib.meld_sort_u32_noalloc.restype = st
    lib.meld_sort_u32_noalloc.argtypes = [vp, vp, vp, sz, st, vp]
    lib.meld_sort_u32_timed.restype = st
    lib.meld_sort_u32_timed.argtypes = [vp, vp, vp, sz, st, vp, ctypes.POINTER(ctypes.c_float),
                                        sz, ctypes.POINTER(sz)]
    lib.meld_sort_u32_steps.restype = st
    lib.meld_sort_u32_steps.argtypes = [vp, vp, vp, sz, i64, st, vp]
    lib.meld_segmented_sort_u32.restype = st
    lib.meld_segmented_sort_u32.argtypes = [vp, vp, sz, vp, sz, st, vp]
    lib.meld_segmented_sort_u32_staged.restype = st
    lib.meld_segmented_sort_u32_staged.argtypes = [vp, vp, sz, vp, sz, st, st, vp]
    lib.meld_segmented_sort_check.restype = st
    lib.meld_segmented_sort_check.argtypes = [vp, vp]
    lib.meld_probe_region.restype = st
    lib.meld_probe_region.argtypes = [vp, sz, u64, u64, ctypes.POINTER(u64), vp]
    lib.meld_probe_network.restype = st
    lib.meld_probe_network.argtypes = [vp, ctypes.c_uint32, ctypes.POINTER(u64), vp]
    lib.meld_probe_segments.restype = st
    lib.meld_probe_segments.argtypes = [vp, vp, sz, ctypes.POINTER(u64), vp]
    lib.meld_tune.restype = st
    lib.meld_tune.argtypes = [vp, ctypes.c_char_p]
    lib.meld_plan_describe.restype = st
    lib.meld_plan_describe.argtypes = [vp, ctypes.c_char_p, sz]
    lib.meld_sort_plan_describe.restype = st
    lib.meld_sort_plan_describe.argtypes = [vp, sz, ctypes.c_int, st, ctypes.c_char_p, sz]
    dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    lib.meld_tune_choose.restype = ctypes.c_int
    lib.meld_tune_choose.argtypes = [ctypes.c_int, dp, ip, ip, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double]
    lib.meld_set_option.restype = st
    lib.meld_set_option.argtypes = [vp, st, i64]
    lib.meld_divergent_region_f32.restype = st
    lib.meld_divergent_region_f32.argtypes = [vp, vp, vp, sz, vp, sz, u64, u64, Side, Side, st, vp]
    lib.meld_probe_region_gathers.restype = st
    lib.meld_probe_region_gathers.argtypes = [vp, vp, vp, sz, vp, sz, u64, u64, Side, Side, st,
                                              vp]
    lib.meld_merge_sort_u32.restype = st
    lib.meld_merge_sort_u32.argtypes = [vp, vp, sz, i64, st, vp]
    lib.meld_oddeven_sort_buckets_u32.restype = st
    lib.meld_oddeven_sort_buckets_u32.argtypes = [vp, vp, sz, ctypes.c_uint32, i64, st, vp]
    lib.meld_region3_f32.restype = st
    lib.meld_region3_f32.argtypes = [vp, vp, vp, sz, vp, sz, u64, u64, u64, Side, Side, Side, st,
                                     vp]
    lib.meld_region_lanetrips_f32.restype = st
    lib.meld_region_lanetrips_f32.argtypes = [vp, vp, vp, sz, vp, sz, u64, u64, SideRange,
                                              SideRange, st, vp]
    _lib = lib
    return lib


def _check(status: int) -> None:
    if status != OK:
        msg = load_library().meld_last_error().decode(errors="replace")
        raise MeldError(status, msg)


def _stream_handle(device: int, stream) -> int:
    """hipStream_t of ``stream`` (a torch stream, a raw handle, or None for the
    current torch stream of ``device``) as an integer."""
    if stream is None:
        import torch
        stream = torch.cuda.current_stream(device)
    return int(stream.cuda_stream if hasattr(stream, "cuda_stream") else stream)


def new_context(device: int):
    """A fresh library context on ``device``, owned by the caller (free it with
    ``destroy_context``); the functions below take it as ``ctx=``."""
    lib = load_library()
    ctx = ctypes.c_void_p()
    _check(lib.meld_create(device, ctypes.byref(ctx)))
    for opt, val in _options.get(device, {}).items():
        _check(lib.meld_set_option(ctx, opt, val))
    return ctx


def destroy_context(ctx) -> None:
    load_library().meld_destroy(ctx)


def context(device: int, stream=None):
    """The library context of (``device``, ``stream``), created on first use; stream
    None is the current torch stream of the device."""
    key = (device, _stream_handle(device, stream))
    with _lock:
        ctx = _ctxs.get(key)
        if ctx is None:
            ctx = new_context(device)
            _ctxs[key] = ctx
        return ctx


def _variant(v) -> int:
    try:
        return _VARIANTS[v]
    except KeyError:
        raise ValueError(f"unknown variant {v!r}") from None


def _launch_args(t, stream, ctx):
    """(context, stream) of a call on tensor t's device: ctx if given, else the
    context of (device, stream)."""
    dev = t.device.index
    h = _stream_handle(dev, stream)
    return (ctx if ctx is not None else context(dev, h)), ctypes.c_void_p(h)


def _u32_tensor(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype not in (torch.uint32, torch.int32) or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous uint32/int32 tensor")
    return t


def sort(keys, payload=None, variant=AUTO, stream=None, ctx=None, noalloc=False):
    """In-place ascending bitonic sort of ``keys`` (u32 bits), moving ``payload`` along.
    noalloc: through meld_sort_u32_noalloc (no device allocation; padding in the
    library's fixed device scratch)."""
    _u32_tensor(keys, "keys")
    if payload is not None:
        _u32_tensor(payload, "payload")
        if payload.numel() != keys.numel() or payload.device != keys.device:
            raise ValueError("payload must match keys in length and device")
    c, s = _launch_args(keys, stream, ctx)
    lib = load_library()
    fn = lib.meld_sort_u32_noalloc if noalloc else lib.meld_sort_u32
    _check(fn(
        c, ctypes.c_void_p(keys.data_ptr()),
        None if payload is None else ctypes.c_void_p(payload.data_ptr()), keys.numel(),
        _variant(variant), s))
    return keys if payload is None else (keys, payload)


def sort_timed(keys, payload=None, variant=AUTO, stream=None, ctx=None) -> list[float]:
    """``sort`` with the duration in ms of each of its launches (HIP events on the
    launch stream, see meld_sort_u32_timed); waits for the sort."""
    _u32_tensor(keys, "keys")
    if payload is not None:
        _u32_tensor(payload, "payload")
        if payload.numel() != keys.numel() or payload.device != keys.device:
            raise ValueError("payload must match keys in length and device")
    c, s = _launch_args(keys, stream, ctx)
    cap = 1024
    out = (ctypes.c_float * cap)()
    n_out = ctypes.c_size_t(0)
    _check(load_library().meld_sort_u32_timed(
        c, ctypes.c_void_p(keys.data_ptr()),
        None if payload is None else ctypes.c_void_p(payload.data_ptr()), keys.numel(),
        _variant(variant), s, out, cap, ctypes.byref(n_out)))
    return [float(out[i]) for i in range(n_out.value)]


def sort_steps(keys, payload=None, max_steps=-1, variant=AUTO, stream=None, ctx=None):
    """The first ``max_steps`` steps of the sorting network (power-of-two length)."""
    _u32_tensor(keys, "keys")
    if payload is not None:
        _u32_tensor(payload, "payload")
    c, s = _launch_args(keys, stream, ctx)
    _check(load_library().meld_sort_u32_steps(
        c, ctypes.c_void_p(keys.data_ptr()),
        None if payload is None else ctypes.c_void_p(payload.data_ptr()), keys.numel(),
        int(max_steps), _variant(variant), s))
    return keys if payload is None else (keys, payload)


def segmented_sort(keys, offsets, variant=AUTO, stream=None, low=None, high=None, ctx=None):
    """Sorts every segment keys[offsets[s]:offsets[s+1]] in place.

    ``low`` / ``high`` pick the form per stage (phases k <= 64 / k >= 128);
    when either is given the other defaults to ``variant``."""
    _u32_tensor(keys, "keys")
    _u32_tensor(offsets, "offsets")
    if offsets.device != keys.device:
        raise ValueError("keys and offsets must be on the same device")
    nseg = max(offsets.numel() - 1, 0)
    if keys.numel() == 0 or nseg == 0:
        return keys
    lib = load_library()
    c, s = _launch_args(keys, stream, ctx)
    args = (c, ctypes.c_void_p(keys.data_ptr()), keys.numel(),
            ctypes.c_void_p(offsets.data_ptr()), nseg)
    if low is None and high is None:
        _check(lib.meld_segmented_sort_u32(*args, _variant(variant), s))
    else:
        lo = _variant(variant if low is None else low)
        hi = _variant(variant if high is None else high)
        _check(lib.meld_segmented_sort_u32_staged(*args, lo, hi, s))
    return keys


def segmented_sort_check(device: int = 0, stream=None, ctx=None):
    """Raises MeldError if a segmented sort on the context of (``device``, ``stream``)
    (or on ``ctx``) met invalid offsets."""
    h = _stream_handle(device, stream)
    c = ctx if ctx is not None else context(device, h)
    _check(load_library().meld_segmented_sort_check(c, ctypes.c_void_p(h)))


OPT_USE_GRAPHS = 0
OPT_SORT_LOG_TILE = 1
OPT_LANE_EXCHANGE = 2


def set_option(device: int, option: int, value: int) -> None:
    """Sets a context option (see meld_set_option) on every context of ``device``,
    present and future."""
    lib = load_library()
    with _lock:
        current = [c for (d, _), c in _ctxs.items() if d == device]
    if not current:
        current = [context(device)]
    for c in current:
        _check(lib.meld_set_option(c, int(option), int(value)))
    _options.setdefault(device, {})[int(option)] = int(value)


def side(a: float, off: int, step: int, trips: int) -> Side:
    return Side(float(a), int(off), int(step), int(trips))


def _as_side(s) -> Side:
    if isinstance(s, Side):
        return s
    return side(s["a"], s["off"], s["step"], s["trips"])


def _region_tensors(x, tab, out):
    import torch
    for t, name in ((x, "x"), (tab, "tab")):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 \
                or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    return torch.empty_like(x) if out is None else out


def divergent_region(x, tab, seed: int, thr: int, side_true, side_false, variant=AUTO,
                     out=None, stream=None, ctx=None, gathers_only=False):
    """Two-sided loop region over the lanes of ``x`` (see meld_divergent_region_f32).
    gathers_only: the form's memory path alone (meld_probe_region_gathers)."""
    out = _region_tensors(x, tab, out)
    c, s = _launch_args(x, stream, ctx)
    lib = load_library()
    fn = lib.meld_probe_region_gathers if gathers_only else lib.meld_divergent_region_f32
    _check(fn(
        c, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), x.numel(),
        ctypes.c_void_p(tab.data_ptr()), tab.numel(), int(seed), int(thr),
        _as_side(side_true), _as_side(side_false), _variant(variant), s))
    return out


def oddeven_sort_buckets(keys, log_bucket: int, max_steps: int = -1, variant=AUTO,
                         stream=None, ctx=None):
    """Sorts each bucket of 2^log_bucket keys in place with Batcher's odd-even merge
    network (see meld_oddeven_sort_buckets_u32)."""
    _u32_tensor(keys, "keys")
    c, s = _launch_args(keys, stream, ctx)
    _check(load_library().meld_oddeven_sort_buckets_u32(
        c, ctypes.c_void_p(keys.data_ptr()), keys.numel(), int(log_bucket), int(max_steps),
        _variant(variant), s))


def merge_sort(keys, max_passes: int = -1, variant=AUTO, stream=None, ctx=None):
    """Ascending bottom-up merge sort of ``keys`` in place (see meld_merge_sort_u32)."""
    _u32_tensor(keys, "keys")
    c, s = _launch_args(keys, stream, ctx)
    _check(load_library().meld_merge_sort_u32(
        c, ctypes.c_void_p(keys.data_ptr()), keys.numel(), int(max_passes), _variant(variant),
        s))


def region3(x, tab, seed: int, thr0: int, thr1: int, way0, way1, way2, variant=AUTO, out=None,
            stream=None, ctx=None):
    """Three-way region over the lanes of ``x`` (see meld_region3_f32)."""
    out = _region_tensors(x, tab, out)
    c, s = _launch_args(x, stream, ctx)
    _check(load_library().meld_region3_f32(
        c, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), x.numel(),
        ctypes.c_void_p(tab.data_ptr()), tab.numel(), int(seed), int(thr0), int(thr1),
        _as_side(way0), _as_side(way1), _as_side(way2), _variant(variant), s))
    return out


def _as_side_range(s) -> SideRange:
    if isinstance(s, SideRange):
        return s
    return SideRange(float(s["a"]), int(s["off"]), int(s["step"]), int(s["trips_lo"]),
                     int(s["trips_hi"]))


def region_lanetrips(x, tab, seed: int, thr: int, side_true, side_false, variant=AUTO,
                     out=None, stream=None, ctx=None):
    """Two-sided region with per-lane trip counts (see meld_region_lanetrips_f32); the
    sides are dicts with a, off, step, trips_lo, trips_hi."""
    out = _region_tensors(x, tab, out)
    c, s = _launch_args(x, stream, ctx)
    _check(load_library().meld_region_lanetrips_f32(
        c, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), x.numel(),
        ctypes.c_void_p(tab.data_ptr()), tab.numel(), int(seed), int(thr),
        _as_side_range(side_true), _as_side_range(side_false), _variant(variant), s))
    return out


def _dev_args(device: int, stream, ctx):
    h = _stream_handle(device, stream)
    return (ctx if ctx is not None else context(device, h)), ctypes.c_void_p(h)


def probe_region(n: int, seed: int, thr: int, device: int = 0, stream=None, ctx=None):
    """(mixed waves, true lanes, waves) of the region branch over lanes [0, n)."""
    out = (ctypes.c_uint64 * 3)()
    c, s = _dev_args(device, stream, ctx)
    _check(load_library().meld_probe_region(c, n, seed, thr, out, s))
    return tuple(int(v) for v in out)


def probe_network(log_t: int, device: int = 0, stream=None, ctx=None):
    """[(mixed comparator-waves, comparator-waves) for phases k = 2 .. 2^log_t]."""
    out = (ctypes.c_uint64 * (2 * log_t))()
    c, s = _dev_args(device, stream, ctx)
    _check(load_library().meld_probe_network(c, log_t, out, s))
    return [(int(out[2 * i]), int(out[2 * i + 1])) for i in range(log_t)]


def probe_segments(offsets, stream=None, ctx=None):
    """(mixed, all) comparator-steps of the phases k <= 64 and of k >= 128."""
    _u32_tensor(offsets, "offsets")
    out = (ctypes.c_uint64 * 4)()
    c, s = _launch_args(offsets, stream, ctx)
    _check(load_library().meld_probe_segments(c, ctypes.c_void_p(offsets.data_ptr()),
                                              max(offsets.numel() - 1, 0), out, s))
    return (int(out[0]), int(out[1])), (int(out[2]), int(out[3]))


def tune(cache_path: str, device: int = 0, stream=None, ctx=None) -> None:
    """Attaches a JSON tuning cache (loads it if present, saves new decisions) to the
    context of (``device``, ``stream``)."""
    c, _ = _dev_args(device, stream, ctx)
    _check(load_library().meld_tune(c, cache_path.encode()))


def plan_describe(device: int = 0, stream=None, ctx=None) -> str:
    """The tuning decisions of the context of (``device``, ``stream``) as JSON text."""
    lib = load_library()
    c, _ = _dev_args(device, stream, ctx)
    size = 1 << 16
    while True:
        buf = ctypes.create_string_buffer(size)
        st = lib.meld_plan_describe(c, buf, size)
        if st == OK:
            return buf.value.decode()
        if size >= 1 << 26:
            _check(st)
        size *= 4


def sort_plan(n: int, pairs: bool = False, variant: str = "auto", device=None, stream=None,
              ctx=None) -> dict:
    """The launches a sort of n elements runs (tile, forms, HBM passes), as a
    dict; device None (and no ctx): the library's default rule without a context."""
    import json
    lib = load_library()
    c = ctx if ctx is not None else (None if device is None else _dev_args(device, stream,
                                                                           None)[0])
    buf = ctypes.create_string_buffer(1 << 16)
    _check(lib.meld_sort_plan_describe(c, n, 1 if pairs else 0, _variant(variant), buf,
                                       len(buf)))
    return json.loads(buf.value.decode())


def tune_choose(ms, melded_lo, melded_hi, mixed_lo, mixed_hi, theta=0.5, tie=0.02) -> int:
    """The tuner's decision rule (pure host function)."""
    n = len(ms)
    return int(load_library().meld_tune_choose(
        n, (ctypes.c_double * n)(*ms), (ctypes.c_int * n)(*melded_lo),
        (ctypes.c_int * n)(*melded_hi), mixed_lo, mixed_hi, theta, tie))
