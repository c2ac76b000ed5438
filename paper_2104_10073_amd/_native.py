"""ctypes binding of libzmc.so (the C ABI declared in include/zmc.h).

Argument marshalling only: every step of the integration runs in the library's
HIP kernels.  There is no fallback: if the library is missing this module
raises, it never computes anything itself.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from .workloads import FUNC_DTYPE

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libzmc.so")

MC_OK = 0
MC_NOT_READY = 1
STATUS_NAMES = {
    0: "MC_OK", 1: "MC_NOT_READY", -1: "MC_ERR_INVALID_ARG", -2: "MC_ERR_UNSUPPORTED_FAMILY",
    -3: "MC_ERR_BAD_DIM", -4: "MC_ERR_BAD_BOUNDS", -5: "MC_ERR_BAD_PARAMS", -6: "MC_ERR_OUT_OF_MEMORY",
    -7: "MC_ERR_ADMISSION", -8: "MC_ERR_HIP", -9: "MC_ERR_NO_DEVICE", -10: "MC_ERR_ABORTED",
    -11: "MC_ERR_UNKNOWN_REQUEST", -12: "MC_ERR_COMPILE",
}

PREC_FP32 = 0
PREC_FP64 = 1

MC_VALIDATE_ONLY = 0x1
MC_NO_GRAPH = 0x2
MC_NO_PROMOTE = 0x4
MC_RESIDENT = 0x8          # serve through one resident kernel (include/zmc.h)
MC_SCHED_FAIR = 0
MC_SCHED_FIFO = 1
MC_SCHED_SRPT = 2
GRID_AXIS_DTYPE = np.dtype([("param", "<u4"), ("count", "<u4"), ("start", "<f8"), ("step", "<f8")])
MC_MAX_GRID_AXES = 4
MC_FAMILY_USER0 = 16        # first run-time family id (mc_register_family)
MC_MAX_USER_FAMILIES = 8

RESULT_DTYPE = np.dtype([
    ("mean", "<f8"), ("std_error", "<f8"), ("sum_f", "<f8"), ("sum_f2", "<f8"),
    ("n", "<u8"), ("status", "<i4"), ("precision", "<u4"),
])
assert RESULT_DTYPE.itemsize == 48

# Every symbol include/zmc.h declares.
EXPORTS = [
    "mc_config_init", "mc_workspace_size", "mc_create", "mc_destroy", "mc_submit", "mc_run",
    "mc_poll", "mc_pending", "mc_results", "mc_abort", "mc_integrate_plain_fp64", "mc_get_tuning",
    "mc_set_tuning", "mc_autotune", "mc_last_run_timing", "mc_get_stats", "mc_last_error",
    "mc_segment_samples", "mc_version", "mc_register_family", "mc_submit_grid",
    "mc_sample_points", "mc_integrate_plain_fp64_noalloc", "mc_snapshot", "mc_restore", "mc_cancel",
]


class McConfig(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("max_functions", ctypes.c_uint32),
        ("max_tiles_per_run", ctypes.c_uint32),
        ("max_partials", ctypes.c_uint64),
        ("mem_budget_bytes", ctypes.c_uint64),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_uint64),
        ("blocks_per_cu", ctypes.c_uint32),
        ("policy", ctypes.c_uint32),
    ]


class McStats(ctypes.Structure):
    _fields_ = [
        ("launches", ctypes.c_uint64), ("tiles32", ctypes.c_uint64), ("tiles64", ctypes.c_uint64),
        ("functions", ctypes.c_uint64), ("samples", ctypes.c_uint64), ("promoted", ctypes.c_uint64),
        ("bad_records", ctypes.c_uint64), ("fp32_ms", ctypes.c_double), ("fp64_ms", ctypes.c_double),
        ("finalize_ms", ctypes.c_double), ("graph_ms", ctypes.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class McError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libzmc.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()' or python paper_2104_10073_amd/build.py)")
    # One HIP runtime per process: PyTorch ships its own libamdhip64 (same soname),
    # and its streams and memory are only valid in that runtime.  Loading torch
    # first makes libzmc.so bind to it instead of starting a second runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(path)
    vp, u64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)
    L.mc_config_init.argtypes = [ctypes.POINTER(McConfig)]
    L.mc_workspace_size.argtypes = [ctypes.POINTER(McConfig), u64p]
    L.mc_create.argtypes = [ctypes.POINTER(McConfig), ctypes.POINTER(vp)]
    L.mc_destroy.argtypes = [vp]
    L.mc_submit.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int32, u64p]
    L.mc_run.argtypes = [vp, vp]
    L.mc_poll.argtypes = [vp, u64p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
    L.mc_pending.argtypes = [vp, u64p, u64p]
    L.mc_results.argtypes = [vp, ctypes.c_uint64, vp, ctypes.c_size_t, ctypes.c_int]
    L.mc_abort.argtypes = [vp]
    L.mc_snapshot.argtypes = [vp, ctypes.c_uint64, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
    L.mc_restore.argtypes = [vp, vp, ctypes.c_size_t, u64p]
    L.mc_cancel.argtypes = [vp, ctypes.c_uint64]
    L.mc_integrate_plain_fp64.argtypes = [vp, vp, ctypes.c_size_t, vp, vp]
    L.mc_integrate_plain_fp64_noalloc.argtypes = [vp, vp, ctypes.c_size_t, vp, vp]
    L.mc_get_tuning.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32), vp]
    L.mc_set_tuning.argtypes = [vp, ctypes.c_uint32, vp]
    L.mc_autotune.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_double]
    L.mc_last_run_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.mc_get_stats.argtypes = [vp, ctypes.POINTER(McStats)]
    L.mc_last_error.argtypes = [vp]
    L.mc_sample_points.argtypes = [vp, vp, ctypes.c_uint64, ctypes.c_uint64, vp, vp]
    L.mc_submit_grid.argtypes = [vp, vp, vp, ctypes.c_uint32, ctypes.c_int32, u64p]
    L.mc_register_family.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_uint32)]
    L.mc_last_error.restype = ctypes.c_char_p
    L.mc_segment_samples.restype = ctypes.c_uint32
    L.mc_version.restype = ctypes.c_char_p
    for name in EXPORTS:
        fn = getattr(L, name)
        if fn.restype is ctypes.c_int:  # default restype: mc_status
            fn.restype = ctypes.c_int
    _lib = L
    return L


def _stream_handle(stream) -> int | None:
    """A hipStream_t as an integer: None (null stream), an int, or a torch.cuda.Stream."""
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    handle = getattr(stream, "cuda_stream", None)
    if handle is None:
        raise TypeError(f"cannot use {stream!r} as a HIP stream")
    return int(handle)


def as_table(fns) -> np.ndarray:
    t = np.ascontiguousarray(fns)
    if t.dtype != FUNC_DTYPE:
        raise TypeError(f"function table must have dtype workloads.FUNC_DTYPE, got {t.dtype}")
    return t


class Context:
    """One mc_ctx.  Device memory comes from the library or, with
    ``workspace='torch'``, from a torch tensor the context keeps alive."""

    def __init__(self, device: int = 0, flags: int = 0, max_functions: int = 0, max_tiles_per_run: int = 0,
                 max_partials: int = 0, mem_budget_bytes: int = 0, workspace=None, blocks_per_cu: int = 0,
                 policy: int = MC_SCHED_FAIR):
        self.L = load()
        cfg = McConfig()
        self.L.mc_config_init(ctypes.byref(cfg))
        cfg.device = device
        cfg.flags = flags
        cfg.max_functions = max_functions
        cfg.max_tiles_per_run = max_tiles_per_run
        cfg.max_partials = max_partials
        cfg.mem_budget_bytes = mem_budget_bytes
        cfg.blocks_per_cu = blocks_per_cu
        cfg.policy = policy
        self._workspace = None
        if workspace is not None:
            need = ctypes.c_uint64()
            self._check(self.L.mc_workspace_size(ctypes.byref(cfg), ctypes.byref(need)), None)
            if isinstance(workspace, str) and workspace == "torch":
                import torch
                workspace = torch.empty(int(need.value) + 256, dtype=torch.uint8, device=f"cuda:{device}")
            ptr = int(workspace.data_ptr())
            pad = (-ptr) % 256
            cfg.workspace = ptr + pad
            cfg.workspace_bytes = int(workspace.numel() * workspace.element_size()) - pad
            self._workspace = workspace
        h = ctypes.c_void_p()
        self._check(self.L.mc_create(ctypes.byref(cfg), ctypes.byref(h)), None)
        self.h = h
        self.config = cfg

    def _check(self, st: int, h) -> int:
        if st < 0:
            msg = self.L.mc_last_error(h)
            raise McError(st, msg.decode() if msg else "")
        return st

    def close(self):
        """mc_destroy: wait for outstanding work and free the context."""
        if getattr(self, "h", None):
            self.L.mc_destroy(self.h)
            self.h = None
        self._workspace = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- batched path
    def submit(self, fns, precision: int = PREC_FP32) -> int:
        """mc_submit: validate and queue a table (numpy FUNC_DTYPE array) as one request; returns its id."""
        t = as_table(fns)
        rid = ctypes.c_uint64()
        self._check(self.L.mc_submit(self.h, t.ctypes.data, len(t), precision, ctypes.byref(rid)), self.h)
        return int(rid.value)

    def submit_grid(self, base, axes, precision: int = PREC_FP32) -> int:
        """Submit `base` (one table row) over a parameter grid; axes = [(param, count, start, step), ...]
        (axis 0 varies fastest).  The request holds prod(count) functions."""
        b = as_table(np.atleast_1d(base))
        if len(b) != 1:
            raise ValueError("base must be a single function")
        ax = np.zeros(len(axes), dtype=GRID_AXIS_DTYPE)
        for i, (param, count, start, step) in enumerate(axes):
            ax[i] = (param, count, start, step)
        rid = ctypes.c_uint64()
        self._check(self.L.mc_submit_grid(self.h, b.ctypes.data, ax.ctypes.data, len(ax), precision,
                                          ctypes.byref(rid)), self.h)
        return int(rid.value)

    def integrate_grid(self, base, axes, precision: int = PREC_FP32, stream=None):
        """submit_grid, one mc_run on `stream`, then the blocking results (prod(count) of them)."""
        n = int(np.prod([a[1] for a in axes]))
        rid = self.submit_grid(base, axes, precision)
        self.run(stream)
        return self.results(rid, n, blocking=True)

    def run(self, stream=None) -> bool:
        """Enqueue one launch; False when every launch slot is still busy (nothing launched)."""
        return self._check(self.L.mc_run(self.h, _stream_handle(stream)), self.h) == MC_OK

    def poll(self, cap: int = 4096):
        """Ids of requests completed since the previous poll."""
        ids = (ctypes.c_uint64 * cap)()
        n = ctypes.c_size_t()
        self._check(self.L.mc_poll(self.h, ids, cap, ctypes.byref(n)), self.h)
        return [int(ids[i]) for i in range(n.value)]

    def validate_tiles(self) -> int:
        """Tiles that the submitted, not yet launched work would take (works on any context)."""
        return self.pending()[1]

    def pending(self):
        """mc_pending: (requests not yet complete, tiles still waiting for a launch)."""
        r, t = ctypes.c_uint64(), ctypes.c_uint64()
        self._check(self.L.mc_pending(self.h, ctypes.byref(r), ctypes.byref(t)), self.h)
        return int(r.value), int(t.value)

    def results(self, request_id: int, n: int, blocking: bool = True, allow_aborted: bool = False):
        """mc_results: the n results of a request (RESULT_DTYPE); None if not blocking and not ready."""
        out = np.zeros(n, dtype=RESULT_DTYPE)
        st = self.L.mc_results(self.h, request_id, out.ctypes.data, n, 1 if blocking else 0)
        if st == MC_NOT_READY:
            return None
        if st == -10 and allow_aborted:
            return out
        self._check(st, self.h)
        return out

    def integrate(self, fns, precision: int = PREC_FP32, stream=None):
        """submit, one mc_run on `stream`, then the blocking results."""
        t = as_table(fns)
        rid = self.submit(t, precision)
        self.run(stream)
        return self.results(rid, len(t), blocking=True)

    def abort(self):
        """mc_abort: stop the running persistent kernels; queued requests complete as aborted."""
        self._check(self.L.mc_abort(self.h), self.h)

    def cancel(self, request_id: int):
        """mc_cancel: drop one request's remaining work; it completes as aborted (results already in stay)."""
        self._check(self.L.mc_cancel(self.h, request_id), self.h)

    def snapshot(self, request_id: int) -> bytes:
        """mc_snapshot: the request's state (results in, tiling, progress, partials of the tiles run)."""
        need = ctypes.c_size_t()
        self._check(self.L.mc_snapshot(self.h, request_id, None, 0, ctypes.byref(need)), self.h)
        buf = ctypes.create_string_buffer(need.value)
        self._check(self.L.mc_snapshot(self.h, request_id, buf, need.value, ctypes.byref(need)), self.h)
        return buf.raw[:need.value]

    def restore(self, blob: bytes) -> int:
        """mc_restore: queue a snapshotted request; returns its new id."""
        rid = ctypes.c_uint64()
        data = ctypes.create_string_buffer(bytes(blob), len(blob))
        self._check(self.L.mc_restore(self.h, data, len(blob), ctypes.byref(rid)), self.h)
        return int(rid.value)

    def register_family(self, source: str) -> int:
        """Compile an integrand family from source (see mc_register_family); returns its family id."""
        fam = ctypes.c_uint32()
        self._check(self.L.mc_register_family(self.h, source.encode(), ctypes.byref(fam)), self.h)
        return int(fam.value)

    def sample_points(self, fn, first: int, count: int, stream=None) -> np.ndarray:
        """Points of samples [first, first + count) of one function, shape (count, dim)."""
        t = as_table(np.atleast_1d(fn))
        if len(t) != 1:
            raise ValueError("one function")
        out = np.zeros((count, int(t["dim"][0])), dtype=np.float64)
        self._check(self.L.mc_sample_points(self.h, t.ctypes.data, first, count, out.ctypes.data,
                                            _stream_handle(stream)), self.h)
        return out

    # -- plain baseline
    def plain_fp64(self, fns, stream=None):
        """mc_integrate_plain_fp64: the one-launch-per-function FP64 comparator (synchronous)."""
        t = as_table(fns)
        out = np.zeros(len(t), dtype=RESULT_DTYPE)
        self._check(self.L.mc_integrate_plain_fp64(self.h, t.ctypes.data, len(t), out.ctypes.data,
                                                   _stream_handle(stream)), self.h)
        return out

    def plain_fp64_noalloc(self, fns, stream=None):
        """mc_integrate_plain_fp64_noalloc: the plain FP64 path with its working set in the
        library's fixed per-GPU array (no device allocation; synchronous)."""
        t = as_table(fns)
        out = np.zeros(len(t), dtype=RESULT_DTYPE)
        self._check(self.L.mc_integrate_plain_fp64_noalloc(self.h, t.ctypes.data, len(t), out.ctypes.data,
                                                           _stream_handle(stream)), self.h)
        return out

    # -- tuning
    def get_tuning(self):
        """mc_get_tuning: (workgroups per CU, seg_log2 array [precision][family][dim - 1])."""
        b = ctypes.c_uint32()
        seg = np.zeros((2, 4, 12), dtype=np.uint8)
        self._check(self.L.mc_get_tuning(self.h, ctypes.byref(b), seg.ctypes.data), self.h)
        return int(b.value), seg

    def set_tuning(self, blocks_per_cu: int = 0, seg_log2=None):
        """mc_set_tuning: 0 / None keep the current value."""
        ptr = None
        if seg_log2 is not None:
            seg = np.ascontiguousarray(seg_log2, dtype=np.uint8).reshape(2, 4, 12)
            ptr = seg.ctypes.data
        self._check(self.L.mc_set_tuning(self.h, blocks_per_cu, ptr), self.h)

    def autotune(self, precision: int = PREC_FP32, stream=None, budget_seconds: float = 10.0):
        """mc_autotune: time candidate tunings on synthetic batches and keep the fastest."""
        self._check(self.L.mc_autotune(self.h, precision, _stream_handle(stream), budget_seconds), self.h)

    def stats(self) -> dict:
        """mc_get_stats: cumulative counters of the context."""
        st = McStats()
        self._check(self.L.mc_get_stats(self.h, ctypes.byref(st)), self.h)
        return st.as_dict()

    def last_run_timing(self):
        """mc_last_run_timing: (persistent kernels ms, finalize and publish ms) of the last direct launch."""
        a, b = ctypes.c_double(), ctypes.c_double()
        st = self.L.mc_last_run_timing(self.h, ctypes.byref(a), ctypes.byref(b))
        if st != MC_OK:
            return None
        return a.value, b.value


def segment_samples() -> int:
    return int(load().mc_segment_samples())


def version() -> str:
    return load().mc_version().decode()
