"""Python binding of libsde, the MI355X (gfx950) SDE-ensemble library.

A thin ctypes layer over the C ABI declared in include/sde.h: each function
here has the name of the C entry point it calls and only marshals arguments
(torch tensors or raw integers become device pointers, Python dicts become
the descriptor structs).  All computation happens in libsde's HIP kernels.
PyTorch is only a source of device memory and streams.

The models are those of Januszewski & Kostur (arXiv:0903.3852): the noisy
driven Josephson junction (Eq. 1) and the noisy Kuramoto model (Eq. 2),
integrated with the stochastic Heun scheme (Alg. 2) or Euler-Maruyama.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libsde.so")

SDE_OK, SDE_ERR_INVALID, SDE_ERR_NOMEM, SDE_ERR_DEVICE, SDE_ERR_UNSUPPORTED, SDE_ERR_NUMERIC = \
    0, -1, -2, -3, -4, -5
SDE_HEUN, SDE_EULER = 0, 1
SDE_INIT_PHILOX, SDE_INIT_FROM_STATE = 0, 1
SDE_MEANFIELD, SDE_TILED, SDE_DENSE_FP32, SDE_DENSE_BF16X3, SDE_DENSE_FP16X3 = 0, 1, 2, 3, 4
SDE_TAG_NOISE, SDE_TAG_INIT = 0, 1
SDE_POTENTIAL_SIN, SDE_POTENTIAL_SIN2PI = 0, 1
SDE_OBS_MEAN_F32, SDE_OBS_MEAN_F64, SDE_OBS_MEANSQ_F32, SDE_OBS_ORDER = 0, 1, 2, 3
SDE_OPT_AUTOTUNE, SDE_OPT_GRAPHS, SDE_OPT_JJ_PPT, SDE_OPT_KURA_MF, SDE_OPT_KURA_JSPLIT, SDE_OPT_KURA_TILE = \
    1, 2, 3, 4, 5, 6
SDE_OPT_KURA_XCD_LOCAL = 7
SDE_OPT_KURA_MF_OPT = 8
SDE_OPT_DENSE_LAUNCH = 9
SDE_OPT_KURA_MF_PAIRED = 10

EXPORTS = ["sde_create", "sde_destroy", "sde_strerror", "sde_last_error", "sde_check",
           "sde_jj_integrate", "sde_jj_integrate_noalloc", "sde_jj_integrate_f64", "sde_jj_integrate_recorded",
           "sde_kuramoto_integrate",
           "sde_observables", "sde_position_histogram", "sde_position_histograms", "sde_phase_histograms",
           "sde_debug_philox", "sde_debug_gauss", "sde_set_option", "sde_set_tune_cache",
           "sde_get_stats", "sde_surrogate_create", "sde_surrogate_destroy",
           "sde_surrogate_param_count", "sde_surrogate_set_params", "sde_surrogate_get_params",
           "sde_surrogate_set_scaling", "sde_surrogate_get_scaling", "sde_surrogate_train",
           "sde_surrogate_predict", "sde_surrogate_loss_grad", "sde_surrogate_scan",
           "sde_surrogate_save", "sde_surrogate_load"]


class SDEError(RuntimeError):
    def __init__(self, status, detail):
        super().__init__(f"{_strerror(status)} ({status}): {detail}")
        self.status = status


class sde_jj_point(ctypes.Structure):
    _fields_ = [("m", ctypes.c_double), ("gamma", ctypes.c_double), ("a", ctypes.c_double),
                ("omega", ctypes.c_double), ("f", ctypes.c_double), ("D", ctypes.c_double),
                ("n_paths", ctypes.c_uint32), ("steps_per_period", ctypes.c_uint32),
                ("n_steps", ctypes.c_uint64), ("n_transient", ctypes.c_uint64),
                ("potential", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class sde_run(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("step0", ctypes.c_uint64), ("scheme", ctypes.c_int32),
                ("init", ctypes.c_int32), ("sample_every", ctypes.c_uint32),
                ("sync", ctypes.c_int32)]


class sde_stats(ctypes.Structure):
    _fields_ = [("graph_replayed", ctypes.c_int32), ("tuned", ctypes.c_int32),
                ("jj_paths_per_lane", ctypes.c_int32), ("graphs_cached", ctypes.c_int32),
                ("tune_ms", ctypes.c_double), ("work_items", ctypes.c_uint64),
                ("mf_streamed", ctypes.c_int32), ("kura_jsplit", ctypes.c_int32),
                ("kura_tile", ctypes.c_int32), ("kura_mf_opt", ctypes.c_int32),
                ("dense_waves", ctypes.c_int32), ("dense_xcd_bands", ctypes.c_int32),
                ("kura_mf_paired", ctypes.c_int32), ("dense_variant", ctypes.c_int32)]


class sde_surrogate_scaling(ctypes.Structure):
    _fields_ = [("in_center", ctypes.c_float * 8), ("in_scale", ctypes.c_float * 8),
                ("out_mean", ctypes.c_float), ("out_std", ctypes.c_float),
                ("target_over_omega", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class sde_train_opts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_uint32), ("batch", ctypes.c_uint32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("shuffle_seed", ctypes.c_uint64)]


class sde_scan_stats(ctypes.Structure):
    _fields_ = [("n_queries", ctypes.c_uint64), ("n_fallback", ctypes.c_uint64),
                ("predict_ms", ctypes.c_double), ("fallback_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double)]


class sde_kuramoto_desc(ctypes.Structure):
    _fields_ = [("N", ctypes.c_uint32), ("R", ctypes.c_uint32), ("K", ctypes.c_double),
                ("D", ctypes.c_double), ("dt", ctypes.c_double), ("n_steps", ctypes.c_uint64),
                ("coupling", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None


def lib():
    """The loaded libsde.so.  Raises if the HIP library has not been built:
    there is no fallback implementation."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise ImportError(f"{LIBPATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIBPATH)
        vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        L.sde_create.argtypes = [i32, ctypes.POINTER(vp)]
        L.sde_create.restype = i32
        L.sde_destroy.argtypes = [vp]
        L.sde_destroy.restype = None
        L.sde_strerror.argtypes = [i32]
        L.sde_strerror.restype = ctypes.c_char_p
        L.sde_last_error.argtypes = [vp]
        L.sde_last_error.restype = ctypes.c_char_p
        L.sde_check.argtypes = [vp]
        L.sde_check.restype = i32
        L.sde_jj_integrate.argtypes = [vp, ctypes.POINTER(sde_jj_point), u32, ctypes.POINTER(sde_run),
                                       vp, vp, vp, vp, vp, vp]
        L.sde_jj_integrate.restype = i32
        L.sde_jj_integrate_noalloc.argtypes = L.sde_jj_integrate.argtypes
        L.sde_jj_integrate_noalloc.restype = i32
        L.sde_jj_integrate_f64.argtypes = [vp, ctypes.POINTER(sde_jj_point), u32, ctypes.POINTER(sde_run),
                                           vp, vp, vp, vp, vp, vp]
        L.sde_jj_integrate_f64.restype = i32
        L.sde_jj_integrate_recorded.argtypes = [vp, ctypes.POINTER(sde_jj_point), u32, ctypes.POINTER(sde_run),
                                                vp, vp, vp, vp, vp, u32, u64, vp, vp]
        L.sde_jj_integrate_recorded.restype = i32
        L.sde_kuramoto_integrate.argtypes = [vp, ctypes.POINTER(sde_kuramoto_desc),
                                             ctypes.POINTER(sde_run), vp, vp, vp, vp, vp]
        L.sde_kuramoto_integrate.restype = i32
        L.sde_observables.argtypes = [vp, i32, vp, ctypes.POINTER(u32), u32,
                                      ctypes.POINTER(ctypes.c_double), vp]
        L.sde_observables.restype = i32
        L.sde_position_histogram.argtypes = [vp, vp, u64, ctypes.c_int64, u32, vp, vp]
        L.sde_position_histogram.restype = i32
        L.sde_position_histograms.argtypes = [vp, vp, u64, u64, u64, ctypes.c_int64, u32, vp, vp]
        L.sde_position_histograms.restype = i32
        L.sde_phase_histograms.argtypes = [vp, vp, u64, u64, u64, u32, vp, vp]
        L.sde_phase_histograms.restype = i32
        L.sde_debug_philox.argtypes = [vp, u64, u32, u32, u32, u64, u64, vp, vp]
        L.sde_debug_philox.restype = i32
        L.sde_debug_gauss.argtypes = [vp, u64, u32, u32, u32, u64, u64, vp, vp]
        L.sde_debug_gauss.restype = i32
        L.sde_set_option.argtypes = [vp, i32, ctypes.c_int64]
        L.sde_set_option.restype = i32
        L.sde_set_tune_cache.argtypes = [vp, ctypes.c_char_p]
        L.sde_set_tune_cache.restype = i32
        L.sde_get_stats.argtypes = [vp, ctypes.POINTER(sde_stats)]
        L.sde_get_stats.restype = i32
        fp = ctypes.POINTER(ctypes.c_float)
        L.sde_surrogate_create.argtypes = [vp, ctypes.POINTER(u32), u32, u32, u64, ctypes.POINTER(vp)]
        L.sde_surrogate_create.restype = i32
        L.sde_surrogate_destroy.argtypes = [vp]
        L.sde_surrogate_destroy.restype = None
        L.sde_surrogate_param_count.argtypes = [vp]
        L.sde_surrogate_param_count.restype = u64
        L.sde_surrogate_set_params.argtypes = [vp, u32, fp, u64]
        L.sde_surrogate_set_params.restype = i32
        L.sde_surrogate_get_params.argtypes = [vp, u32, fp, u64]
        L.sde_surrogate_get_params.restype = i32
        L.sde_surrogate_set_scaling.argtypes = [vp, ctypes.POINTER(sde_surrogate_scaling)]
        L.sde_surrogate_set_scaling.restype = i32
        L.sde_surrogate_get_scaling.argtypes = [vp, ctypes.POINTER(sde_surrogate_scaling)]
        L.sde_surrogate_get_scaling.restype = i32
        L.sde_surrogate_train.argtypes = [vp, vp, vp, u64, ctypes.POINTER(sde_train_opts), fp, vp]
        L.sde_surrogate_train.restype = i32
        L.sde_surrogate_predict.argtypes = [vp, vp, u64, vp, vp, vp]
        L.sde_surrogate_predict.restype = i32
        L.sde_surrogate_loss_grad.argtypes = [vp, u32, vp, vp, u64, fp, ctypes.POINTER(ctypes.c_double), vp]
        L.sde_surrogate_loss_grad.restype = i32
        L.sde_surrogate_scan.argtypes = [vp, ctypes.POINTER(sde_jj_point), u64, ctypes.c_float,
                                         ctypes.POINTER(sde_run), vp, vp, ctypes.POINTER(sde_scan_stats), vp]
        L.sde_surrogate_scan.restype = i32
        L.sde_surrogate_save.argtypes = [vp, ctypes.c_char_p]
        L.sde_surrogate_save.restype = i32
        L.sde_surrogate_load.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(vp)]
        L.sde_surrogate_load.restype = i32
        _lib = L
    return _lib


def _strerror(status):
    try:
        return lib().sde_strerror(status).decode()
    except ImportError:
        return str(status)


def _ptr(x):
    """Device pointer of a torch tensor / raw int / None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


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


def _check(ctx, status):
    if status != SDE_OK:
        raise SDEError(status, lib().sde_last_error(ctx).decode())
    return status


def sde_create(device=0):
    h = ctypes.c_void_p()
    st = lib().sde_create(device, ctypes.byref(h))
    if st != SDE_OK:
        raise SDEError(st, f"sde_create(device={device})")
    return h.value


def sde_destroy(ctx):
    lib().sde_destroy(ctx)


def sde_strerror(status):
    return lib().sde_strerror(status).decode()


def sde_last_error(ctx):
    return lib().sde_last_error(ctx).decode()


def sde_check(ctx):
    return _check(ctx, lib().sde_check(ctx))


def make_points(params):
    """list of dicts (m, gamma, a, omega, f, D, n_paths, steps_per_period,
    n_steps, n_transient, optionally potential) -> ctypes array of
    sde_jj_point."""
    arr = (sde_jj_point * len(params))()
    for i, p in enumerate(params):
        for k, _ in sde_jj_point._fields_:
            if k == "reserved":
                continue
            setattr(arr[i], k, p.get(k, SDE_POTENTIAL_SIN) if k == "potential" else p[k])
    return arr


JJ_POINT_DTYPE = np.dtype([("m", "<f8"), ("gamma", "<f8"), ("a", "<f8"), ("omega", "<f8"),
                           ("f", "<f8"), ("D", "<f8"), ("n_paths", "<u4"),
                           ("steps_per_period", "<u4"), ("n_steps", "<u8"), ("n_transient", "<u8"),
                           ("potential", "<i4"), ("reserved", "<i4")])


def make_points_np(**cols):
    """Vectorized make_points: keyword arrays (or scalars) for every field
    of sde_jj_point (potential optional, default SDE_POTENTIAL_SIN); returns
    a ctypes array viewing one numpy buffer."""
    n = max(np.size(v) for v in cols.values())
    arr = np.zeros(n, dtype=JJ_POINT_DTYPE)
    for k in JJ_POINT_DTYPE.names:
        if k == "reserved" or (k == "potential" and k not in cols):
            continue
        arr[k] = cols[k]
    out = (sde_jj_point * n).from_buffer(arr)
    out._keep = arr
    return out


def make_run(seed, step0=0, scheme=SDE_HEUN, init=SDE_INIT_PHILOX, sample_every=0, sync=0):
    return sde_run(seed, step0, scheme, init, sample_every, sync)


def sde_jj_integrate(ctx, pts, run, theta=None, winding=None, v=None, acc=None, point_sums=None,
                     stream=None):
    """pts: ctypes array from make_points (or a list of dicts); run: sde_run."""
    if not isinstance(pts, ctypes.Array):
        pts = make_points(pts)
    return _check(ctx, lib().sde_jj_integrate(ctx, pts, len(pts), ctypes.byref(run), _ptr(theta),
                                              _ptr(winding), _ptr(v), _ptr(acc), _ptr(point_sums),
                                              _stream(stream)))


def sde_jj_integrate_noalloc(ctx, pts, run, theta=None, winding=None, v=None, acc=None, point_sums=None,
                             stream=None):
    """As sde_jj_integrate, through the entry point that allocates nothing
    (static device scratch of the library)."""
    if not isinstance(pts, ctypes.Array):
        pts = make_points(pts)
    return _check(ctx, lib().sde_jj_integrate_noalloc(ctx, pts, len(pts), ctypes.byref(run), _ptr(theta),
                                                      _ptr(winding), _ptr(v), _ptr(acc), _ptr(point_sums),
                                                      _stream(stream)))


def sde_jj_integrate_f64(ctx, pts, run, theta=None, winding=None, v=None, acc=None, point_sums=None,
                         stream=None):
    """As sde_jj_integrate, with float64 theta and v."""
    if not isinstance(pts, ctypes.Array):
        pts = make_points(pts)
    return _check(ctx, lib().sde_jj_integrate_f64(ctx, pts, len(pts), ctypes.byref(run), _ptr(theta),
                                                  _ptr(winding), _ptr(v), _ptr(acc), _ptr(point_sums),
                                                  _stream(stream)))


def sde_jj_integrate_recorded(ctx, pts, run, record_every, rec_winding, theta=None, winding=None, v=None,
                              acc=None, point_sums=None, stream=None):
    """sde_jj_integrate that writes every path's winding every record_every
    steps into the device int32 tensor rec_winding [n_rows, total paths]."""
    if not isinstance(pts, ctypes.Array):
        pts = make_points(pts)
    n_rows = rec_winding.shape[0] if rec_winding is not None and rec_winding.dim() == 2 else 0
    return _check(ctx, lib().sde_jj_integrate_recorded(ctx, pts, len(pts), ctypes.byref(run), _ptr(theta),
                                                       _ptr(winding), _ptr(v), _ptr(acc), _ptr(point_sums),
                                                       int(record_every), int(n_rows), _ptr(rec_winding),
                                                       _stream(stream)))


def sde_kuramoto_integrate(ctx, desc, run, phi, omega, K=None, r_samples=None, stream=None):
    return _check(ctx, lib().sde_kuramoto_integrate(ctx, ctypes.byref(desc), ctypes.byref(run),
                                                    _ptr(phi), _ptr(omega), _ptr(K),
                                                    _ptr(r_samples), _stream(stream)))


def sde_observables(ctx, kind, dev_in, counts, stream=None):
    """Returns a float64 numpy array [n_groups, 2]."""
    counts = np.ascontiguousarray(counts, dtype=np.uint32)
    out = np.zeros((len(counts), 2), dtype=np.float64)
    _check(ctx, lib().sde_observables(ctx, kind, _ptr(dev_in),
                                      counts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                      len(counts),
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      _stream(stream)))
    return out


def sde_position_histogram(ctx, winding, x0, n_bins, counts, stream=None):
    """Histogram of a device int32 winding array into device uint64
    counts[n_bins + 2] (underflow, bins x0 .. x0 + n_bins - 1, overflow)."""
    return _check(ctx, lib().sde_position_histogram(ctx, _ptr(winding), int(winding.numel()), int(x0),
                                                    int(n_bins), _ptr(counts), _stream(stream)))


def sde_position_histograms(ctx, winding, x0, n_bins, counts, n=None, stream=None):
    """Row-wise histograms of a device int32 tensor winding [n_rows, pitch]
    (the first n entries of each row, default all) into device uint64
    counts [n_rows, n_bins + 2]."""
    n_rows, pitch = winding.shape
    n = pitch if n is None else n
    return _check(ctx, lib().sde_position_histograms(ctx, _ptr(winding), int(n), int(winding.stride(0)),
                                                     int(n_rows), int(x0), int(n_bins), _ptr(counts),
                                                     _stream(stream)))


def sde_phase_histograms(ctx, theta, n_bins, counts, n=None, stream=None):
    """Row-wise phase histograms of a device float32 tensor theta [n_rows,
    pitch] (revolutions; the first n entries of each row, default all) into
    device uint64 counts [n_rows, n_bins + 1] (last column: outside [0, 1])."""
    if theta.dim() == 1:
        theta = theta.view(1, -1)
    n_rows, pitch = theta.shape
    n = pitch if n is None else n
    return _check(ctx, lib().sde_phase_histograms(ctx, _ptr(theta), int(n), int(theta.stride(0)), int(n_rows),
                                                  int(n_bins), _ptr(counts), _stream(stream)))


def sde_debug_philox(ctx, seed, tag, a, b, ctr0_first, n_blocks, dev_out, stream=None):
    return _check(ctx, lib().sde_debug_philox(ctx, seed, tag, a, b, ctr0_first, n_blocks,
                                              _ptr(dev_out), _stream(stream)))


def sde_debug_gauss(ctx, seed, tag, a, b, n_first, count, dev_out, stream=None):
    return _check(ctx, lib().sde_debug_gauss(ctx, seed, tag, a, b, n_first, count,
                                             _ptr(dev_out), _stream(stream)))


def sde_set_option(ctx, option, value):
    return _check(ctx, lib().sde_set_option(ctx, option, value))


def sde_set_tune_cache(ctx, path):
    return _check(ctx, lib().sde_set_tune_cache(ctx, None if path is None else str(path).encode()))


def sde_get_stats(ctx):
    """dict of the last integration call's launch statistics."""
    st = sde_stats()
    _check(ctx, lib().sde_get_stats(ctx, ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in sde_stats._fields_}


# ---- surrogate ---------------------------------------------------------------
# A surrogate handle is (ctx, pointer): errors are reported through its context.
def sde_surrogate_create(ctx, widths, n_members, seed):
    w = (ctypes.c_uint32 * len(widths))(*widths)
    h = ctypes.c_void_p()
    _check(ctx, lib().sde_surrogate_create(ctx, w, len(widths), n_members, seed, ctypes.byref(h)))
    return (ctx, h.value)


def sde_surrogate_destroy(s):
    lib().sde_surrogate_destroy(s[1])


def sde_surrogate_param_count(s):
    return int(lib().sde_surrogate_param_count(s[1]))


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def sde_surrogate_set_params(s, member, params):
    p = np.ascontiguousarray(params, dtype=np.float32)
    return _check(s[0], lib().sde_surrogate_set_params(s[1], member, _fptr(p), p.size))


def sde_surrogate_get_params(s, member):
    p = np.empty(sde_surrogate_param_count(s), dtype=np.float32)
    _check(s[0], lib().sde_surrogate_get_params(s[1], member, _fptr(p), p.size))
    return p


def make_scaling(in_center, in_scale, out_mean=0.0, out_std=1.0, target_over_omega=0):
    sc = sde_surrogate_scaling()
    for i in range(8):
        sc.in_center[i] = in_center[i] if i < len(in_center) else 0.0
        sc.in_scale[i] = in_scale[i] if i < len(in_scale) else 1.0
    sc.out_mean, sc.out_std, sc.target_over_omega, sc.reserved = out_mean, out_std, target_over_omega, 0
    return sc


def sde_surrogate_set_scaling(s, sc):
    return _check(s[0], lib().sde_surrogate_set_scaling(s[1], ctypes.byref(sc)))


def sde_surrogate_get_scaling(s):
    sc = sde_surrogate_scaling()
    _check(s[0], lib().sde_surrogate_get_scaling(s[1], ctypes.byref(sc)))
    return sc


def make_train_opts(epochs, batch, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, shuffle_seed=0):
    return sde_train_opts(epochs, batch, lr, beta1, beta2, eps, shuffle_seed)


def sde_surrogate_train(s, X, y, opts, stream=None, loss_curve=True):
    """Returns the per-epoch loss curve (numpy) or None."""
    n = X.shape[0]
    curve = np.zeros(opts.epochs, dtype=np.float32) if loss_curve else None
    _check(s[0], lib().sde_surrogate_train(s[1], _ptr(X), _ptr(y), n, ctypes.byref(opts),
                                           _fptr(curve) if curve is not None else None,
                                           _stream(stream)))
    return curve


def sde_surrogate_predict(s, X, mean, spread, stream=None):
    return _check(s[0], lib().sde_surrogate_predict(s[1], _ptr(X), X.shape[0], _ptr(mean),
                                                    _ptr(spread), _stream(stream)))


def sde_surrogate_loss_grad(s, member, X, y, stream=None):
    """(loss, packed gradient as float32 numpy)."""
    g = np.empty(sde_surrogate_param_count(s), dtype=np.float32)
    loss = ctypes.c_double()
    _check(s[0], lib().sde_surrogate_loss_grad(s[1], member, _ptr(X), _ptr(y), X.shape[0], _fptr(g),
                                               ctypes.byref(loss), _stream(stream)))
    return loss.value, g


def sde_surrogate_scan(s, queries, spread_max, fallback_run, v_out, used_fallback=None, stream=None):
    """queries: list of dicts or ctypes array; returns the scan statistics dict."""
    if not isinstance(queries, ctypes.Array):
        queries = make_points(queries)
    st = sde_scan_stats()
    _check(s[0], lib().sde_surrogate_scan(s[1], queries, len(queries), spread_max,
                                          ctypes.byref(fallback_run), _ptr(v_out), _ptr(used_fallback),
                                          ctypes.byref(st), _stream(stream)))
    return {k: getattr(st, k) for k, _ in sde_scan_stats._fields_}


def sde_surrogate_save(s, path):
    return _check(s[0], lib().sde_surrogate_save(s[1], str(path).encode()))


def sde_surrogate_load(ctx, path):
    h = ctypes.c_void_p()
    _check(ctx, lib().sde_surrogate_load(ctx, str(path).encode(), ctypes.byref(h)))
    return (ctx, h.value)
