"""ctypes binding of libcjt_hip.so (C-ABI in include/cjt.h), same names.

Argument marshalling only: every step of the transform runs in the HIP
library.  Device buffers are passed as torch tensors (float64, contiguous, on
the GPU) or as raw integer device addresses; streams as torch.cuda.Stream,
raw hipStream_t integers, or None for torch's current stream.

The library must have been built (`python -m paper_1602_02618_amd.build`);
there is no fallback: if it is missing, loading raises.
"""
import ctypes
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcjt_hip.so")

CJT_OK, CJT_EINVAL, CJT_EDOMAIN, CJT_ENOMEM, CJT_EDEVICE, CJT_EBUSY, CJT_EUNSUPPORTED, CJT_ECANCELED = range(8)
CJT_FP64 = 0
CJT_FP32_BULK = 1
CJT_BATCH_INVARIANT = 8
CJT_SHIFT = 16
CJT_DIR_FWD = 2
CJT_DIR_INV = 4
CJT_MAX_BLOCKS = 16

_EXPORTS = (
    "cjt_plan", "cjt_forward", "cjt_inverse", "cjt_forward_batched", "cjt_inverse_batched",
    "cjt_jacobi_to_jacobi", "cjt_jacobi_to_jacobi_batched",
    "cjt_plan_query", "cjt_plan_describe", "cjt_plan_destroy", "cjt_strerror", "cjt_last_error",
    "cjt_version", "cjt_profile_enable", "cjt_profile_collect",
    "cjt_batch_create", "cjt_batch_execute", "cjt_batch_query", "cjt_batch_destroy",
    "cjt_server_create", "cjt_server_submit", "cjt_server_replay", "cjt_server_wait", "cjt_server_cancel",
    "cjt_server_pause", "cjt_server_drain", "cjt_server_query", "cjt_server_destroy",
    "cjt_autotune", "cjt_tune_set", "cjt_tune_save", "cjt_tune_load",
)


class cjt_partition_info(ctypes.Structure):
    _fields_ = [
        ("grid", ctypes.c_int64),
        ("M", ctypes.c_int32),
        ("nblocks", ctypes.c_int32),
        ("n_M", ctypes.c_int64),
        ("alpha_N", ctypes.c_double),
        ("K", ctypes.c_int32),
        ("theta_bar", ctypes.c_int32),
        ("deg_lo", ctypes.c_int64 * CJT_MAX_BLOCKS),
        ("deg_hi", ctypes.c_int64 * CJT_MAX_BLOCKS),
        ("win_lo", ctypes.c_int64 * CJT_MAX_BLOCKS),
        ("win_hi", ctypes.c_int64 * CJT_MAX_BLOCKS),
        ("rec_entries", ctypes.c_int64),
    ]

    def blocks(self):
        """[(deg_lo, deg_hi, win_lo, win_hi), ...] for the nblocks Hahn blocks."""
        return [(self.deg_lo[k], self.deg_hi[k], self.win_lo[k], self.win_hi[k]) for k in range(self.nblocks)]


class cjt_kernel_stat(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 48),
        ("launches", ctypes.c_int64),
        ("total_ms", ctypes.c_double),
        ("flops", ctypes.c_double),
        ("bytes", ctypes.c_double),
    ]


class cjt_plan_info(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64),
        ("alpha", ctypes.c_double),
        ("beta", ctypes.c_double),
        ("M", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("eps", ctypes.c_double),
        ("fwd", cjt_partition_info),
        ("inv", cjt_partition_info),
        ("fft_len_fwd", ctypes.c_int64),
        ("fft_len_inv", ctypes.c_int64),
        ("fft_count_fwd", ctypes.c_int64),
        ("fft_count_inv", ctypes.c_int64),
        ("device_bytes", ctypes.c_size_t),
        ("fft_log2_cols_fwd", ctypes.c_int32),
        ("fft_log2_cols_inv", ctypes.c_int32),
        ("shift_alpha", ctypes.c_int32),
        ("shift_beta", ctypes.c_int32),
    ]


class cjt_batch_info(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_int64),
        ("launches", ctypes.c_int64),
        ("items", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_size_t),
        ("inverse", ctypes.c_int32),
    ]


class cjt_server_config(ctypes.Structure):
    _fields_ = [
        ("hbm_budget", ctypes.c_size_t),
        ("workspace_bytes", ctypes.c_size_t),
        ("max_batch", ctypes.c_int32),
        ("max_inflight", ctypes.c_int32),
        ("M", ctypes.c_int32),
        ("start_paused", ctypes.c_int32),
    ]


class cjt_server_stats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64),
        ("completed", ctypes.c_int64),
        ("failed", ctypes.c_int64),
        ("cancelled", ctypes.c_int64),
        ("batches", ctypes.c_int64),
        ("mean_batch", ctypes.c_double),
        ("plan_hits", ctypes.c_int64),
        ("plan_misses", ctypes.c_int64),
        ("plan_evictions", ctypes.c_int64),
        ("admission_stalls", ctypes.c_int64),
        ("plans_resident", ctypes.c_int64),
        ("plan_bytes", ctypes.c_size_t),
        ("budget_bytes", ctypes.c_size_t),
        ("peak_used_bytes", ctypes.c_size_t),
        ("lat_count", ctypes.c_int64),
        ("lat_p50_us", ctypes.c_double),
        ("lat_p99_us", ctypes.c_double),
        ("lat_mean_us", ctypes.c_double),
        ("lat_max_us", ctypes.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class cjt_tune_entry(ctypes.Structure):
    _fields_ = [
        ("fft_len", ctypes.c_int64),
        ("inverse", ctypes.c_int32),
        ("chirp", ctypes.c_int32),
        ("fp32", ctypes.c_int32),
        ("candidates", ctypes.c_int32),
        ("log2_cols_default", ctypes.c_int32),
        ("log2_cols_best", ctypes.c_int32),
        ("ms_default", ctypes.c_double),
        ("ms_best", ctypes.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class CJTError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what}: {_strerror(status)} ({status}): {_last_error()}")


_lock = threading.Lock()
_lib = None


def load(path=LIB_PATH):
    """Open libcjt_hip.so (once) and declare its signatures."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError(f"HIP library {path} is not built; run `python -m paper_1602_02618_amd.build`")
        lib = ctypes.CDLL(path)
        vp, i64, dbl, ci, cu = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int, ctypes.c_uint
        P = ctypes.POINTER
        lib.cjt_plan.argtypes = [P(vp), i64, dbl, dbl, ci, cu, vp]
        lib.cjt_forward.argtypes = [vp, vp, vp, vp]
        lib.cjt_inverse.argtypes = [vp, vp, vp, vp]
        lib.cjt_forward_batched.argtypes = [P(vp), i64, P(i64), vp, vp, vp]
        lib.cjt_inverse_batched.argtypes = [P(vp), i64, P(i64), vp, vp, vp]
        lib.cjt_jacobi_to_jacobi.argtypes = [vp, vp, vp, vp, vp]
        lib.cjt_jacobi_to_jacobi_batched.argtypes = [P(vp), P(vp), i64, P(i64), vp, vp, vp]
        lib.cjt_plan_query.argtypes = [vp, P(cjt_plan_info)]
        lib.cjt_plan_describe.argtypes = [i64, dbl, dbl, ci, cu, P(cjt_plan_info)]
        lib.cjt_plan_destroy.argtypes = [vp]
        lib.cjt_strerror.argtypes = [ci]
        lib.cjt_strerror.restype = ctypes.c_char_p
        lib.cjt_last_error.argtypes = []
        lib.cjt_last_error.restype = ctypes.c_char_p
        lib.cjt_version.argtypes = []
        lib.cjt_version.restype = ci
        lib.cjt_profile_enable.argtypes = [ci]
        lib.cjt_profile_enable.restype = ci
        lib.cjt_profile_collect.argtypes = [P(cjt_kernel_stat), ci, P(ci)]
        lib.cjt_profile_collect.restype = ci
        lib.cjt_batch_create.argtypes = [P(vp), P(vp), i64, P(i64), cu, vp]
        lib.cjt_batch_execute.argtypes = [vp, vp, vp, vp]
        lib.cjt_batch_query.argtypes = [vp, P(cjt_batch_info)]
        lib.cjt_batch_destroy.argtypes = [vp]
        lib.cjt_server_create.argtypes = [P(vp), P(cjt_server_config)]
        lib.cjt_server_submit.argtypes = [vp, cu, i64, dbl, dbl, vp, vp, P(i64)]
        lib.cjt_server_replay.argtypes = [vp, i64, P(cu), P(i64), P(dbl), P(dbl), P(vp), P(vp), P(dbl), P(i64)]
        lib.cjt_server_wait.argtypes = [vp, i64, P(ci), P(dbl)]
        lib.cjt_server_cancel.argtypes = [vp, i64]
        lib.cjt_server_pause.argtypes = [vp, ci]
        lib.cjt_server_drain.argtypes = [vp]
        lib.cjt_server_query.argtypes = [vp, P(cjt_server_stats), ci]
        lib.cjt_server_destroy.argtypes = [vp]
        lib.cjt_autotune.argtypes = [i64, cu, i64, ci, vp, P(cjt_tune_entry), P(ci)]
        lib.cjt_tune_set.argtypes = [i64, ci, ci, ci, ci]
        lib.cjt_tune_save.argtypes = [ctypes.c_char_p]
        lib.cjt_tune_load.argtypes = [ctypes.c_char_p]
        for f in ("cjt_autotune", "cjt_tune_set", "cjt_tune_save", "cjt_tune_load"):
            getattr(lib, f).restype = ci
        for f in ("cjt_plan", "cjt_forward", "cjt_inverse", "cjt_forward_batched", "cjt_inverse_batched",
                  "cjt_plan_query", "cjt_plan_describe", "cjt_plan_destroy", "cjt_batch_create",
                  "cjt_batch_execute", "cjt_batch_query", "cjt_batch_destroy", "cjt_server_create",
                  "cjt_server_submit", "cjt_server_replay", "cjt_server_wait", "cjt_server_cancel",
                  "cjt_server_pause", "cjt_server_drain", "cjt_server_query", "cjt_server_destroy"):
            getattr(lib, f).restype = ci
        _lib = lib
        return lib


def _strerror(st):
    return load().cjt_strerror(int(st)).decode()


def _last_error():
    return load().cjt_last_error().decode()


def _check(st, what):
    if st != CJT_OK:
        raise CJTError(st, what)


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    # torch tensor on the GPU, float64, contiguous
    if getattr(x, "dtype", None) is not None:
        import torch
        if x.dtype != torch.float64 or not x.is_contiguous() or not x.is_cuda:
            raise ValueError("device buffers must be contiguous float64 GPU tensors")
        return x.data_ptr()
    raise TypeError(f"cannot pass {type(x)!r} as a device pointer")


def _stream(s):
    if s is None:
        try:
            import torch
            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except ImportError:
            pass
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


class Plan:
    """Owning wrapper of a cjt_plan_t."""

    def __init__(self, handle):
        self.handle = handle

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def destroy(self):
        if self.handle:
            h, self.handle = self.handle, None
            load().cjt_plan_destroy(h)

    @property
    def info(self):
        return cjt_plan_query(self)

    @property
    def N(self):
        return self.info.N


def cjt_plan(N, alpha, beta, M=0, flags=CJT_FP64, stream=None):
    h = ctypes.c_void_p()
    _check(load().cjt_plan(ctypes.byref(h), int(N), float(alpha), float(beta), int(M), int(flags), _stream(stream)),
           "cjt_plan")
    return Plan(h.value)


def cjt_forward(plan, d_in, d_out, stream=None):
    _check(load().cjt_forward(plan.handle, _ptr(d_in), _ptr(d_out), _stream(stream)), "cjt_forward")


def cjt_inverse(plan, d_in, d_out, stream=None):
    _check(load().cjt_inverse(plan.handle, _ptr(d_in), _ptr(d_out), _stream(stream)), "cjt_inverse")


def _batched(fn, what, plans, offsets, d_in, d_out, stream):
    n = len(plans)
    arr = (ctypes.c_void_p * max(n, 1))(*[p.handle for p in plans])
    offs = (ctypes.c_int64 * (n + 1))(*[int(o) for o in offsets])
    _check(fn(arr, n, offs, _ptr(d_in), _ptr(d_out), _stream(stream)), what)


def cjt_forward_batched(plans, offsets, d_in, d_out, stream=None):
    _batched(load().cjt_forward_batched, "cjt_forward_batched", plans, offsets, d_in, d_out, stream)


def cjt_inverse_batched(plans, offsets, d_in, d_out, stream=None):
    _batched(load().cjt_inverse_batched, "cjt_inverse_batched", plans, offsets, d_in, d_out, stream)


def cjt_jacobi_to_jacobi(src, dst, d_in, d_out, stream=None):
    _check(load().cjt_jacobi_to_jacobi(src.handle, dst.handle, _ptr(d_in), _ptr(d_out), _stream(stream)),
           "cjt_jacobi_to_jacobi")


def cjt_jacobi_to_jacobi_batched(src, dst, offsets, d_in, d_out, stream=None):
    n = len(src)
    a = (ctypes.c_void_p * max(n, 1))(*[p.handle for p in src])
    b = (ctypes.c_void_p * max(len(dst), 1))(*[p.handle for p in dst])
    if len(dst) != n:
        raise ValueError("source and target plan lists differ in length")
    offs = (ctypes.c_int64 * (n + 1))(*[int(o) for o in offsets])
    _check(load().cjt_jacobi_to_jacobi_batched(a, b, n, offs, _ptr(d_in), _ptr(d_out), _stream(stream)),
           "cjt_jacobi_to_jacobi_batched")


class Batch:
    """Owning wrapper of a cjt_batch_t; keeps its plans alive."""

    def __init__(self, handle, plans):
        self.handle = handle
        self.plans = list(plans)

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def destroy(self):
        if self.handle:
            h, self.handle = self.handle, None
            load().cjt_batch_destroy(h)

    @property
    def info(self):
        return cjt_batch_query(self)


def cjt_batch_create(plans, offsets, flags, stream=None):
    n = len(plans)
    arr = (ctypes.c_void_p * max(n, 1))(*[p.handle for p in plans])
    offs = (ctypes.c_int64 * (n + 1))(*[int(o) for o in offsets])
    h = ctypes.c_void_p()
    _check(load().cjt_batch_create(ctypes.byref(h), arr, n, offs, int(flags), _stream(stream)), "cjt_batch_create")
    return Batch(h.value, plans)


def cjt_batch_execute(batch, d_in, d_out, stream=None):
    _check(load().cjt_batch_execute(batch.handle, _ptr(d_in), _ptr(d_out), _stream(stream)), "cjt_batch_execute")


def cjt_batch_query(batch):
    info = cjt_batch_info()
    _check(load().cjt_batch_query(batch.handle, ctypes.byref(info)), "cjt_batch_query")
    return info


def cjt_batch_destroy(batch):
    batch.destroy()


class Server:
    """Owning wrapper of a cjt_server_t (continuous-batching transform server)."""

    def __init__(self, handle):
        self.handle = handle

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def destroy(self):
        if self.handle:
            h, self.handle = self.handle, None
            load().cjt_server_destroy(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def submit(self, flags, N, alpha, beta, d_in, d_out):
        return cjt_server_submit(self, flags, N, alpha, beta, d_in, d_out)

    def wait(self, ticket):
        return cjt_server_wait(self, ticket)

    def stats(self, reset=False):
        return cjt_server_query(self, reset)


def cjt_server_create(hbm_budget, workspace_bytes=0, max_batch=0, max_inflight=0, M=0, start_paused=False):
    cfg = cjt_server_config(int(hbm_budget), int(workspace_bytes), int(max_batch), int(max_inflight), int(M),
                            1 if start_paused else 0)
    h = ctypes.c_void_p()
    _check(load().cjt_server_create(ctypes.byref(h), ctypes.byref(cfg)), "cjt_server_create")
    return Server(h.value)


def cjt_server_submit(server, flags, N, alpha, beta, d_in, d_out):
    """Queue one request; returns its ticket.  d_in must be ready (synchronise its producer first)."""
    t = ctypes.c_int64(-1)
    _check(load().cjt_server_submit(server.handle, int(flags), int(N), float(alpha), float(beta), _ptr(d_in),
                                    _ptr(d_out), ctypes.byref(t)), "cjt_server_submit")
    return t.value


def cjt_server_replay(server, flags, N, alpha, beta, d_in, d_out, arrival_us):
    """Submit request i at arrival_us[i] microseconds after the call starts; returns the tickets."""
    n = len(flags)
    A = lambda ct, xs: (ct * max(n, 1))(*xs)
    tickets = (ctypes.c_int64 * max(n, 1))()
    _check(load().cjt_server_replay(server.handle, n, A(ctypes.c_uint, [int(f) for f in flags]),
                                    A(ctypes.c_int64, [int(x) for x in N]), A(ctypes.c_double, [float(x) for x in alpha]),
                                    A(ctypes.c_double, [float(x) for x in beta]),
                                    A(ctypes.c_void_p, [_ptr(x) for x in d_in]),
                                    A(ctypes.c_void_p, [_ptr(x) for x in d_out]),
                                    A(ctypes.c_double, [float(x) for x in arrival_us]), tickets),
           "cjt_server_replay")
    return [tickets[i] for i in range(n)]


def cjt_server_wait(server, ticket):
    """Block until the request completes; returns (status, latency_us)."""
    st = ctypes.c_int(0)
    lat = ctypes.c_double(0.0)
    _check(load().cjt_server_wait(server.handle, int(ticket), ctypes.byref(st), ctypes.byref(lat)), "cjt_server_wait")
    return st.value, lat.value


def cjt_server_cancel(server, ticket):
    """Returns the status: CJT_OK if cancelled, CJT_EBUSY if already running."""
    return int(load().cjt_server_cancel(server.handle, int(ticket)))


def cjt_server_pause(server, paused=True):
    _check(load().cjt_server_pause(server.handle, 1 if paused else 0), "cjt_server_pause")


def cjt_server_drain(server):
    _check(load().cjt_server_drain(server.handle), "cjt_server_drain")


def cjt_server_query(server, reset=False):
    out = cjt_server_stats()
    _check(load().cjt_server_query(server.handle, ctypes.byref(out), 1 if reset else 0), "cjt_server_query")
    return out


def cjt_server_destroy(server):
    server.destroy()


def cjt_autotune(N, flags=CJT_FP64, batch=1, reps=3, stream=None):
    """Time the two-pass splits of a plan of degree N (batched calls of `batch`
    transforms) and keep the fastest; returns the entries."""
    arr = (cjt_tune_entry * 2)()
    n = ctypes.c_int(0)
    _check(load().cjt_autotune(int(N), int(flags), int(batch), int(reps), _stream(stream), arr, ctypes.byref(n)),
           "cjt_autotune")
    return [arr[i] for i in range(n.value)]


def cjt_tune_set(fft_len, inverse, chirp, fp32, log2_cols):
    _check(load().cjt_tune_set(int(fft_len), int(inverse), int(chirp), int(fp32), int(log2_cols)), "cjt_tune_set")


def cjt_tune_save(path):
    _check(load().cjt_tune_save(os.fsencode(path)), "cjt_tune_save")


def cjt_tune_load(path):
    _check(load().cjt_tune_load(os.fsencode(path)), "cjt_tune_load")


def cjt_plan_query(plan):
    info = cjt_plan_info()
    _check(load().cjt_plan_query(plan.handle, ctypes.byref(info)), "cjt_plan_query")
    return info


def cjt_plan_describe(N, alpha, beta, M=0, flags=CJT_FP64):
    info = cjt_plan_info()
    _check(load().cjt_plan_describe(int(N), float(alpha), float(beta), int(M), int(flags), ctypes.byref(info)),
           "cjt_plan_describe")
    return info


def cjt_plan_destroy(plan):
    plan.destroy()


def cjt_strerror(status):
    return _strerror(status)


def cjt_last_error():
    return _last_error()


def cjt_version():
    return int(load().cjt_version())


def cjt_profile_enable(on=True):
    _check(load().cjt_profile_enable(1 if on else 0), "cjt_profile_enable")


def cjt_profile_collect(max_entries=64):
    """{name: dict(launches, total_ms, flops, bytes)} of the kernels timed since the last collect."""
    arr = (cjt_kernel_stat * max_entries)()
    n = ctypes.c_int(0)
    _check(load().cjt_profile_collect(arr, max_entries, ctypes.byref(n)), "cjt_profile_collect")
    return {arr[i].name.decode(): dict(launches=arr[i].launches, total_ms=arr[i].total_ms, flops=arr[i].flops,
                                       bytes=arr[i].bytes) for i in range(n.value)}


# ---------------------------------------------------------------- conveniences

def forward(plan, x, stream=None):
    """Allocate and return the forward transform of the GPU tensor x."""
    import torch
    out = torch.empty_like(x)
    cjt_forward(plan, x, out, stream)
    return out


def inverse(plan, x, stream=None):
    """Allocate and return the inverse transform of the GPU tensor x."""
    import torch
    out = torch.empty_like(x)
    cjt_inverse(plan, x, out, stream)
    return out


def jacobi_to_jacobi(src, dst, x, stream=None):
    """Allocate and return the coefficients in dst's parameters of the
    expansion with coefficients x (GPU tensor) in src's parameters."""
    import torch
    out = torch.empty_like(x)
    cjt_jacobi_to_jacobi(src, dst, x, out, stream)
    return out
