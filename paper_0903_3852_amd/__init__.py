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
SDE_OBS_MEAN_F32, SDE_OBS_MEAN_F64, SDE_OBS_MEANSQ_F32, SDE_OBS_ORDER = 0, 1, 2, 3
SDE_OPT_AUTOTUNE, SDE_OPT_GRAPHS, SDE_OPT_JJ_PPT = 1, 2, 3

EXPORTS = ["sde_create", "sde_destroy", "sde_strerror", "sde_last_error", "sde_check",
           "sde_jj_integrate", "sde_kuramoto_integrate", "sde_observables",
           "sde_debug_philox", "sde_debug_gauss", "sde_set_option", "sde_set_tune_cache",
           "sde_get_stats"]


class SDEError(RuntimeError):
    def __init__(self, status, detail):
        super().__init__(f"{_strerror(status)} ({status}): {detail}")
        self.status = status


class sde_jj_point(ctypes.Structure):
    _fields_ = [("m", ctypes.c_double), ("gamma", ctypes.c_double), ("a", ctypes.c_double),
                ("omega", ctypes.c_double), ("f", ctypes.c_double), ("D", ctypes.c_double),
                ("n_paths", ctypes.c_uint32), ("steps_per_period", ctypes.c_uint32),
                ("n_steps", ctypes.c_uint64), ("n_transient", ctypes.c_uint64)]


class sde_run(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("step0", ctypes.c_uint64), ("scheme", ctypes.c_int32),
                ("init", ctypes.c_int32), ("sample_every", ctypes.c_uint32),
                ("sync", ctypes.c_int32)]


class sde_stats(ctypes.Structure):
    _fields_ = [("graph_replayed", ctypes.c_int32), ("tuned", ctypes.c_int32),
                ("jj_paths_per_lane", ctypes.c_int32), ("graphs_cached", ctypes.c_int32),
                ("tune_ms", ctypes.c_double), ("work_items", ctypes.c_uint64)]


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
        L.sde_kuramoto_integrate.argtypes = [vp, ctypes.POINTER(sde_kuramoto_desc),
                                             ctypes.POINTER(sde_run), vp, vp, vp, vp, vp]
        L.sde_kuramoto_integrate.restype = i32
        L.sde_observables.argtypes = [vp, i32, vp, ctypes.POINTER(u32), u32,
                                      ctypes.POINTER(ctypes.c_double), vp]
        L.sde_observables.restype = i32
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
    n_steps, n_transient) -> ctypes array of sde_jj_point."""
    arr = (sde_jj_point * len(params))()
    for i, p in enumerate(params):
        for k, _ in sde_jj_point._fields_:
            setattr(arr[i], k, p[k])
    return arr


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
