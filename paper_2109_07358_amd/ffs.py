"""ctypes binding of libffs (include/ffs.h) -- argument marshalling only.

Every step of the sampler runs in the library's HIP kernels; this module
converts numpy/torch arguments to pointers and statuses to exceptions.
PyTorch provides device memory and streams.  If libffs.so is missing the
calls raise FFSError: there is no CPU fallback.

Function names mirror the C ABI (ffs_plan, ffs_sample, ffs_marginal, ...).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libffs.so")

FFS_OK = 0
STATUS_NAMES = {0: "FFS_OK", -1: "FFS_ERR_INVALID_ARG",
                -2: "FFS_ERR_NOT_ORTHONORMAL", -3: "FFS_ERR_OUT_OF_MEMORY",
                -4: "FFS_ERR_HIP", -5: "FFS_ERR_NUMERICAL",
                -6: "FFS_ERR_UNSUPPORTED"}
BULK = {"fp64": 0, "fp32": 1, "split_bf16": 2}
PATH = {"batched": 0, "plain": 1}
RESOLVE = {"auto": 0, "per_step": 1, "deferred": 2}

# Every symbol include/ffs.h declares.
EXPORTS = ("ffs_default_options", "ffs_plan", "ffs_sample", "ffs_marginal",
           "ffs_check", "ffs_destroy", "ffs_last_error", "ffs_conditional",
           "ffs_density", "ffs_philox_words", "ffs_set_timing",
           "ffs_set_timing_classes", "ffs_set_timing_stride", "ffs_kernel_times",
           "ffs_server_default_options",
           "ffs_server_create", "ffs_server_submit", "ffs_server_poll",
           "ffs_server_destroy", "ffs_sample_group", "ffs_sample_subsets",
           "ffs_autotune", "ffs_set_tile", "ffs_plan_device", "ffs_dpp_eig",
           "ffs_dpp_subsets", "ffs_kdpp_subsets", "ffs_sample_dpp",
           "ffs_jastrow_estimate", "ffs_sample_mh", "ffs_sample_noalloc",
           "ffs_kernel_spans")
GROUP_GRAPH = 1
REQ_STATES = {0: "queued", 1: "running", 2: "done"}
KERNEL_CLASSES = ("factor", "weights", "draw", "repair", "plain", "factor_block")


class FFSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("bulk", ctypes.c_int32), ("path", ctypes.c_int32),
                ("ortho_tol", ctypes.c_double),
                ("guard_delta", ctypes.c_double),
                ("max_batch", ctypes.c_int64), ("hbm_budget", ctypes.c_size_t),
                ("overlap", ctypes.c_int32), ("resolve", ctypes.c_int32),
                ("guard_scale", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("draws", ctypes.c_int64), ("flagged", ctypes.c_int64),
                ("changed", ctypes.c_int64), ("device_status", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class Instance(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("n_keep", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("first_sample", ctypes.c_uint64),
                ("n_samples", ctypes.c_int64), ("x_dev", ctypes.c_void_p),
                ("logdet_dev", ctypes.c_void_p)]


SERVE_MODES = {"grouped": 0, "streams": 1}


class ServerOptions(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("hbm_budget", ctypes.c_size_t), ("capacity", ctypes.c_int32),
                ("ticks", ctypes.c_int32)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("status", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("draws", ctypes.c_int64),
                ("flagged", ctypes.c_int64), ("changed", ctypes.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["state"] = REQ_STATES.get(d["state"], d["state"])
        return d


_lib = None


def load(path=LIB_PATH):
    """Load libffs.so (once) and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FFSError(-4, "%s not built; run paper_2109_07358_amd.build" % path)
    L = ctypes.CDLL(path)
    vp, i64, u64, i32, dbl = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64,
                              ctypes.c_int32, ctypes.c_double)
    L.ffs_default_options.argtypes = [ctypes.POINTER(Options)]
    L.ffs_default_options.restype = None
    L.ffs_plan.argtypes = [ctypes.POINTER(vp), vp, i64, i64, i64, i32,
                           ctypes.POINTER(Options)]
    L.ffs_plan.restype = ctypes.c_int
    L.ffs_sample.argtypes = [vp, u64, u64, i64, vp, vp, vp]
    L.ffs_sample.restype = ctypes.c_int
    L.ffs_sample_noalloc.argtypes = [vp, u64, u64, i64, vp, vp, vp]
    L.ffs_sample_noalloc.restype = ctypes.c_int
    L.ffs_marginal.argtypes = [vp, i64, u64, u64, i64, vp, vp]
    L.ffs_marginal.restype = ctypes.c_int
    L.ffs_check.argtypes = [vp, ctypes.POINTER(Stats)]
    L.ffs_check.restype = ctypes.c_int
    L.ffs_destroy.argtypes = [vp]
    L.ffs_destroy.restype = ctypes.c_int
    L.ffs_last_error.argtypes = []
    L.ffs_last_error.restype = ctypes.c_char_p
    L.ffs_conditional.argtypes = [vp, u64, u64, i64, vp, vp]
    L.ffs_conditional.restype = ctypes.c_int
    L.ffs_density.argtypes = [vp, vp]
    L.ffs_density.restype = ctypes.c_int
    L.ffs_philox_words.argtypes = [u64, u64, ctypes.c_uint32, vp]
    L.ffs_philox_words.restype = None
    L.ffs_set_timing.argtypes = [vp, i32]
    L.ffs_set_timing.restype = ctypes.c_int
    L.ffs_plan_device.argtypes = [ctypes.POINTER(vp), vp, i64, i64, i64, i32,
                                  ctypes.POINTER(Options)]
    L.ffs_plan_device.restype = ctypes.c_int
    L.ffs_dpp_eig.argtypes = [vp, i64, i64, vp, vp, vp, ctypes.POINTER(ctypes.c_int32), vp]
    L.ffs_dpp_eig.restype = ctypes.c_int
    L.ffs_dpp_subsets.argtypes = [vp, i64, u64, u64, i64, vp, vp, vp]
    L.ffs_dpp_subsets.restype = ctypes.c_int
    L.ffs_kdpp_subsets.argtypes = [vp, i64, i64, u64, u64, i64, vp, vp]
    L.ffs_kdpp_subsets.restype = ctypes.c_int
    L.ffs_sample_dpp.argtypes = [vp, vp, vp, u64, u64, i64, vp, vp, vp]
    L.ffs_sample_dpp.restype = ctypes.c_int
    L.ffs_jastrow_estimate.argtypes = [vp, i64, vp, i64, i64, i64, dbl, vp, vp, vp, vp, vp, vp]
    L.ffs_jastrow_estimate.restype = ctypes.c_int
    L.ffs_sample_mh.argtypes = [vp, i32, i32, u64, u64, i64, vp, vp,
                                ctypes.POINTER(ctypes.c_int64), vp]
    L.ffs_sample_mh.restype = ctypes.c_int
    L.ffs_set_timing_classes.argtypes = [vp, ctypes.c_uint32]
    L.ffs_set_timing_classes.restype = ctypes.c_int
    L.ffs_set_timing_stride.argtypes = [vp, ctypes.c_int32]
    L.ffs_set_timing_stride.restype = ctypes.c_int
    L.ffs_kernel_times.argtypes = [vp, vp, vp]
    L.ffs_kernel_times.restype = ctypes.c_int
    L.ffs_kernel_spans.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
    L.ffs_kernel_spans.restype = ctypes.c_int
    L.ffs_server_default_options.argtypes = [ctypes.POINTER(ServerOptions)]
    L.ffs_server_default_options.restype = None
    L.ffs_server_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(ServerOptions)]
    L.ffs_server_create.restype = ctypes.c_int
    L.ffs_server_submit.argtypes = [vp, vp, i64, u64, u64, i64, vp, vp,
                                    ctypes.POINTER(u64)]
    L.ffs_server_submit.restype = ctypes.c_int
    L.ffs_server_poll.argtypes = [vp, u64, i32, ctypes.POINTER(RequestInfo)]
    L.ffs_server_poll.restype = ctypes.c_int
    L.ffs_server_destroy.argtypes = [vp]
    L.ffs_server_destroy.restype = ctypes.c_int
    L.ffs_set_tile.argtypes = [vp, i64, i32, i32, i32]
    L.ffs_set_tile.restype = ctypes.c_int
    L.ffs_autotune.argtypes = [vp, i64, i32, ctypes.c_char_p]
    L.ffs_autotune.restype = ctypes.c_int
    L.ffs_sample_subsets.argtypes = [vp, i64, vp, u64, u64, i64, vp, vp, vp]
    L.ffs_sample_subsets.restype = ctypes.c_int
    L.ffs_sample_group.argtypes = [ctypes.POINTER(Instance), i32, i32,
                                   ctypes.POINTER(Stats), vp]
    L.ffs_sample_group.restype = ctypes.c_int
    _lib = L
    return L


def ffs_last_error():
    return load().ffs_last_error().decode()


def _check(st):
    if st != FFS_OK:
        raise FFSError(st, ffs_last_error())


def ffs_default_options():
    o = Options()
    load().ffs_default_options(ctypes.byref(o))
    return o


def ffs_philox_words(seed, sample, step):
    out = (ctypes.c_uint32 * 4)()
    load().ffs_philox_words(seed, sample, step, out)
    return tuple(out)


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))


class Plan:
    """An ffs_plan_t for one U (host numpy, float64 or complex128, L x N)."""

    def __init__(self, U, bulk="fp32", path="batched", ortho_tol=None,
                 guard_delta=None, max_batch=None, hbm_budget=None,
                 overlap=None, guard_scale=None, resolve="auto"):
        dev = getattr(U, "is_cuda", False)
        if dev:  # torch cuda tensor, float64 or complex128, row-major
            if U.dim() != 2 or not U.is_contiguous():
                raise ValueError("device U must be a contiguous 2-D tensor")
            cplx = U.is_complex()
            self._host = None
            self._dev = U
            self.L, self.N = U.shape
        else:
            U = np.asarray(U)
            if U.ndim != 2:
                raise ValueError("U must be 2-D")
            cplx = np.iscomplexobj(U)
            self._host = np.ascontiguousarray(U, dtype=np.complex128 if cplx else np.float64)
            self.L, self.N = self._host.shape
        self.cplx = cplx
        o = ffs_default_options()
        o.bulk = BULK[bulk]
        o.path = PATH[path]
        if ortho_tol is not None:
            o.ortho_tol = ortho_tol
        if guard_delta is not None:
            o.guard_delta = guard_delta
        if guard_scale is not None:
            o.guard_scale = guard_scale
        if max_batch is not None:
            o.max_batch = max_batch
        if hbm_budget is not None:
            o.hbm_budget = hbm_budget
        if overlap is not None:
            o.overlap = 1 if overlap else 0
        o.resolve = RESOLVE[resolve]
        self.options = o
        h = ctypes.c_void_p()
        if dev:
            _check(load().ffs_plan_device(ctypes.byref(h), self._dev.data_ptr(),
                                          self.L, self.N, self.N, 1 if cplx else 0,
                                          ctypes.byref(o)))
        else:
            _check(load().ffs_plan(ctypes.byref(h), self._host.ctypes.data,
                                   self.L, self.N, self.N, 1 if cplx else 0,
                                   ctypes.byref(o)))
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise FFSError(-1, "plan destroyed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            load().ffs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ffs_plan(U, **kw):
    return Plan(U, **kw)


def ffs_destroy(plan):
    plan.close()


def _need(t, dtype, numel, name):
    """A caller-supplied device buffer must be a contiguous cuda tensor of
    `dtype` with at least `numel` elements: the library writes through its
    raw pointer, so anything else would be written past its end."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError("%s must be a torch tensor" % name)
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or t.numel() < numel:
        raise ValueError("%s must be a contiguous cuda %s tensor with >= %d elements "
                         "(got %s %s, %d elements%s)"
                         % (name, dtype, numel, t.device, t.dtype, t.numel(),
                            "" if t.is_contiguous() else ", not contiguous"))
    return t


def _out_rows(x_out, n, k, name="x_out"):
    import torch
    if x_out is None:
        return torch.empty((n, k), dtype=torch.int32, device="cuda")
    return _need(x_out, torch.int32, n * k, name)


def ffs_sample(plan, seed, first_sample, n_samples, x_out=None, logdet=False,
               stream=None):
    """Enqueue n_samples draws; returns (x int32 [n, N] cuda, logdet or None)."""
    import torch
    x_out = _out_rows(x_out, n_samples, plan.N)
    ld = torch.empty(n_samples, dtype=torch.float64, device="cuda") if logdet else None
    _check(load().ffs_sample(plan.handle, seed, first_sample, n_samples,
                             x_out.data_ptr(), ld.data_ptr() if ld is not None else None,
                             _stream_ptr(stream)))
    return x_out, ld


def ffs_sample_noalloc(plan, seed, first_sample, n_samples, x_out, logdet_out=None,
                       stream=None):
    """ffs_sample with the library's fixed scratch array as working memory (no
    device allocation in the call): the caller passes the outputs, x_out int32
    cuda [n, N] and optionally logdet_out float64 cuda [n]."""
    import torch
    _need(x_out, torch.int32, n_samples * plan.N, "x_out")
    if logdet_out is not None:
        _need(logdet_out, torch.float64, n_samples, "logdet_out")
    _check(load().ffs_sample_noalloc(plan.handle, seed, first_sample, n_samples,
                                     x_out.data_ptr(),
                                     logdet_out.data_ptr() if logdet_out is not None else None,
                                     _stream_ptr(stream)))
    return x_out, logdet_out


def ffs_marginal(plan, n_keep, seed, first_sample, n_samples, x_out=None,
                 stream=None):
    x_out = _out_rows(x_out, n_samples, n_keep)
    _check(load().ffs_marginal(plan.handle, n_keep, seed, first_sample,
                               n_samples, x_out.data_ptr(), _stream_ptr(stream)))
    return x_out


def ffs_sample_subsets(plan, cols, seed, first_sample, x_out=None, logdet=False,
                       stream=None):
    """Per-sample column subsets: cols int32 cuda [n, k]; returns (x, logdet)."""
    import torch
    n, k = cols.shape
    _need(cols, torch.int32, n * k, "cols")
    x_out = _out_rows(x_out, n, k)
    ld = torch.empty(n, dtype=torch.float64, device="cuda") if logdet else None
    _check(load().ffs_sample_subsets(plan.handle, k, cols.data_ptr(), seed, first_sample,
                                     n, x_out.data_ptr(),
                                     ld.data_ptr() if ld is not None else None,
                                     _stream_ptr(stream)))
    return x_out, ld


def ffs_dpp_eig(B, stream=None):
    """Eigenpairs of B B^T through the dual (B: cuda float64 [L, d]).

    Returns (lam [d] ascending, U [L, d], W [d, d], sweeps), all cuda float64
    except sweeps."""
    import torch
    if not (B.is_cuda and B.dtype == torch.float64 and B.dim() == 2 and B.is_contiguous()):
        raise ValueError("B must be a contiguous cuda float64 matrix")
    L, d = B.shape
    lam = torch.empty(d, dtype=torch.float64, device="cuda")
    U = torch.empty((L, d), dtype=torch.float64, device="cuda")
    W = torch.empty((d, d), dtype=torch.float64, device="cuda")
    sweeps = ctypes.c_int32(0)
    _check(load().ffs_dpp_eig(B.data_ptr(), L, d, lam.data_ptr(), U.data_ptr(),
                              W.data_ptr(), ctypes.byref(sweeps), _stream_ptr(stream)))
    return lam, U, W, sweeps.value


def ffs_dpp_subsets(lam, seed, first_sample, n, stream=None):
    """Eigenvector selection lambda/(lambda+1): (cols [n, d] with -1 padding, sizes [n])."""
    import torch
    d = lam.shape[0]
    _need(lam, torch.float64, d, "lam")
    cols = torch.empty((n, d), dtype=torch.int32, device="cuda")
    sizes = torch.empty(n, dtype=torch.int32, device="cuda")
    _check(load().ffs_dpp_subsets(lam.data_ptr(), d, seed, first_sample, n,
                                  cols.data_ptr(), sizes.data_ptr(), _stream_ptr(stream)))
    return cols, sizes


def ffs_kdpp_subsets(lam, k, seed, first_sample, n, stream=None):
    """Fixed-size eigenvector selection: cols int32 cuda [n, k], ascending."""
    import torch
    d = lam.shape[0]
    _need(lam, torch.float64, d, "lam")
    cols = torch.empty((n, k), dtype=torch.int32, device="cuda")
    _check(load().ffs_kdpp_subsets(lam.data_ptr(), d, k, seed, first_sample, n,
                                   cols.data_ptr(), _stream_ptr(stream)))
    return cols


def ffs_sample_dpp(plan, cols, sizes, seed, first_sample, logdet=False, stream=None):
    """Variable-size subsets (cols [n, N] int32 cuda, sizes [n]): (x [n, N], logdet)."""
    import torch
    n = sizes.shape[0]
    _need(sizes, torch.int32, n, "sizes")
    _need(cols, torch.int32, n * plan.N, "cols")
    x = torch.empty((n, plan.N), dtype=torch.int32, device="cuda")
    ld = torch.empty(n, dtype=torch.float64, device="cuda") if logdet else None
    _check(load().ffs_sample_dpp(plan.handle, cols.data_ptr(), sizes.data_ptr(), seed,
                                 first_sample, n, x.data_ptr(),
                                 ld.data_ptr() if ld is not None else None,
                                 _stream_ptr(stream)))
    return x, ld


JASTROW_SUMMARY = ("D_J", "D_0", "sum_w", "sum_w2", "ess", "shift")


def ffs_jastrow_estimate(x_up, x_dn, L, V, vmat=None, extra_logw=None, stream=None):
    """Reweighted site densities and double occupancy (cuda int32 x rows).

    Returns (logw [n], density [L], summary dict)."""
    import torch
    n, ku = x_up.shape
    kd = x_dn.shape[1] if x_dn is not None else 0
    _need(x_up, torch.int32, n * ku, "x_up")
    if x_dn is not None:
        _need(x_dn, torch.int32, n * kd, "x_dn")
    if vmat is not None:
        _need(vmat, torch.float64, L * L, "vmat")
    if extra_logw is not None:
        _need(extra_logw, torch.float64, n, "extra_logw")
    logw = torch.empty(n, dtype=torch.float64, device="cuda")
    dens = torch.empty(L, dtype=torch.float64, device="cuda")
    summ = torch.empty(6, dtype=torch.float64, device="cuda")
    _check(load().ffs_jastrow_estimate(
        x_up.data_ptr(), ku, x_dn.data_ptr() if x_dn is not None else None, kd, n, L,
        float(V), vmat.data_ptr() if vmat is not None else None,
        extra_logw.data_ptr() if extra_logw is not None else None,
        logw.data_ptr(), dens.data_ptr(), summ.data_ptr(), _stream_ptr(stream)))
    return logw, dens, dict(zip(JASTROW_SUMMARY, summ.cpu().tolist()))


def ffs_sample_mh(plan, m_cond, radius, seed, first_sample, n_samples, x_out=None,
                  logdet=False, accepted=False, stream=None):
    """Metropolis conditional update (large L): (x [n, N], logdet or None, accepted or None)."""
    import torch
    x_out = _out_rows(x_out, n_samples, plan.N)
    ld = torch.empty(n_samples, dtype=torch.float64, device="cuda") if logdet else None
    acc = ctypes.c_int64(0)
    _check(load().ffs_sample_mh(plan.handle, m_cond, radius, seed, first_sample, n_samples,
                                x_out.data_ptr(), ld.data_ptr() if ld is not None else None,
                                ctypes.byref(acc) if accepted else None, _stream_ptr(stream)))
    return x_out, ld, (acc.value if accepted else None)


def ffs_autotune(plan, n_samples, pipeline=False):
    """Time the contraction tile variants for this plan's launches (alone, or
    inside short sampling calls with pipeline=True); returns the choice."""
    buf = ctypes.create_string_buffer(32)
    _check(load().ffs_autotune(plan.handle, n_samples, 1 if pipeline else 0, buf))
    return buf.value.decode()


def ffs_set_tile(plan, n_samples, sites, cols=None, kchunk=0):
    """Record a contraction tile by hand: sites x columns per workgroup and
    the K chunk (0 = 32).  A name "SxC" or "SxCkK" may be given as `sites`."""
    if isinstance(sites, str):
        sites, cols, kchunk = parse_tile(sites)
    _check(load().ffs_set_tile(plan.handle, n_samples, sites, cols, kchunk))


def parse_tile(name):
    """"128x128" -> (128, 128, 32); "128x128k16" -> (128, 128, 16)."""
    head, _, kc = name.partition("k")
    s, c = head.split("x")
    return int(s), int(c), int(kc) if kc else 32


def ffs_check(plan):
    s = Stats()
    _check(load().ffs_check(plan.handle, ctypes.byref(s)))
    return s.as_dict()


def ffs_conditional(plan, seed, sample, prefix):
    k = len(prefix) + 1
    pre = np.ascontiguousarray(np.asarray(prefix, dtype=np.int32))
    out = np.zeros(plan.L)
    _check(load().ffs_conditional(plan.handle, seed, sample, k,
                                  pre.ctypes.data if len(pre) else None,
                                  out.ctypes.data))
    return out


def ffs_set_timing(plan, enable=True):
    _check(load().ffs_set_timing(plan.handle, 1 if enable else 0))


def ffs_set_timing_classes(plan, classes):
    """Time only the launches of the named kernel classes (empty: off)."""
    mask = 0
    for c in classes:
        mask |= 1 << KERNEL_CLASSES.index(c)
    _check(load().ffs_set_timing_classes(plan.handle, ctypes.c_uint32(mask)))


def ffs_set_timing_stride(plan, stride):
    """Time one launch in every `stride` of each timed class."""
    _check(load().ffs_set_timing_stride(plan.handle, int(stride)))


def ffs_kernel_times(plan):
    """{class: (total ms, launches)} since the last read (HIP events)."""
    n = len(KERNEL_CLASSES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    _check(load().ffs_kernel_times(plan.handle, ms, cnt))
    return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNEL_CLASSES)}


def ffs_kernel_spans(plan):
    """(total ms, launches) of the timed contraction launches on the device's
    steady clock (first workgroup start to last workgroup end), since the
    last read."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(load().ffs_kernel_spans(plan.handle, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def ffs_density(plan):
    out = np.zeros(plan.L)
    _check(load().ffs_density(plan.handle, out.ctypes.data))
    return out


def ffs_sample_group(items, graph=True, stats=False, stream=None):
    """Run many instances in lockstep (one launch per phase for all).

    items: list of dicts {plan, n_keep, seed, first_sample, n_samples,
    x_out (int32 cuda [n, n_keep]), logdet_out (optional)}.  Returns the
    per-instance stats list when stats=True, else None."""
    import torch
    n = len(items)
    arr = (Instance * max(n, 1))()
    for it in items:
        _need(it["x_out"], torch.int32, it["n_samples"] * it["n_keep"], "x_out")
        if it.get("logdet_out") is not None:
            _need(it["logdet_out"], torch.float64, it["n_samples"], "logdet_out")
    for i, it in enumerate(items):
        arr[i].plan = it["plan"].handle
        arr[i].n_keep = it["n_keep"]
        arr[i].seed = it["seed"]
        arr[i].first_sample = it["first_sample"]
        arr[i].n_samples = it["n_samples"]
        arr[i].x_dev = it["x_out"].data_ptr()
        ld = it.get("logdet_out")
        arr[i].logdet_dev = ld.data_ptr() if ld is not None else None
    st = (Stats * max(n, 1))() if stats else None
    _check(load().ffs_sample_group(arr, n, GROUP_GRAPH if graph else 0,
                                   st, _stream_ptr(stream)))
    return [st[i].as_dict() for i in range(n)] if stats else None


class Server:
    """An ffs_server_t: requests from any plan run concurrently on its streams."""

    def __init__(self, mode="grouped", slots=None, hbm_budget=None,
                 capacity=None, ticks=None):
        o = ServerOptions()
        load().ffs_server_default_options(ctypes.byref(o))
        o.mode = SERVE_MODES[mode]
        if slots is not None:
            o.slots = slots
        if capacity is not None:
            o.capacity = capacity
        if ticks is not None:
            o.ticks = ticks
        if hbm_budget is not None:
            o.hbm_budget = hbm_budget
        h = ctypes.c_void_p()
        _check(load().ffs_server_create(ctypes.byref(h), ctypes.byref(o)))
        self._h = h
        self.options = o

    def submit(self, plan, n_keep, seed, first_sample, n_samples, x_out,
               logdet_out=None):
        """Queue a request writing x_out (int32 cuda [n, n_keep]); returns its ticket."""
        import torch
        _need(x_out, torch.int32, n_samples * n_keep, "x_out")
        if logdet_out is not None:
            _need(logdet_out, torch.float64, n_samples, "logdet_out")
        t = ctypes.c_uint64()
        _check(load().ffs_server_submit(
            self._h, plan.handle, n_keep, seed, first_sample, n_samples,
            x_out.data_ptr(),
            logdet_out.data_ptr() if logdet_out is not None else None,
            ctypes.byref(t)))
        return t.value

    def poll(self, ticket, timeout_ms=0):
        info = RequestInfo()
        _check(load().ffs_server_poll(self._h, ticket, timeout_ms, ctypes.byref(info)))
        return info.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None:
            load().ffs_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
