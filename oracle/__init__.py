"""FP64 CPU oracle for the SDE ensemble method of Januszewski & Kostur
(arXiv:0903.3852).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product library
never does.  It shares no code with the HIP path: the C part (oracle.c)
restates Philox4x32-10, Box-Muller, the Josephson-junction (Eq. 1) and
Kuramoto (Eq. 2, Eq. 3) drifts and the stochastic Heun step (Alg. 2) from
their definitions, in double precision.

Parity status of each routine:
  philox / gauss          pinned (rocRAND's Philox4x32-10, pure-Python
                          restatement, moment and KS tests)
  jj_integrate            pinned (Boltzmann equilibrium moments with inertia
                          and in the overdamped limit at gamma != 1,
                          overdamped relaxation variance from a well's
                          bottom, overdamped tilted-washboard velocity,
                          order-2 convergence of the deterministic drive)
  ou_integrate            pinned (exact stationary variance of the discrete
                          Heun / Euler schemes, continuum moments)
  kuramoto_integrate      pinned (free diffusion 2Dt, identical-oscillator
                          self-consistency and K_c = 2D, Adler's law, Eq. 3
                          identity between the three coupling forms)
  mlp (oracle.mlp)        pinned (torch CPU reference layers, central finite
                          differences, closed-form first Adam step)
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "liboracle.so")

HEUN, EULER = 0, 1
MEANFIELD, DIRECT, DENSE = 0, 1, 2
TAG_NOISE, TAG_INIT = 0, 1

_lib = None


class JJPoint(ctypes.Structure):
    _fields_ = [("m", ctypes.c_double), ("gamma", ctypes.c_double), ("a", ctypes.c_double),
                ("omega", ctypes.c_double), ("f", ctypes.c_double), ("D", ctypes.c_double),
                ("n_paths", ctypes.c_uint32), ("steps_per_period", ctypes.c_uint32),
                ("n_steps", ctypes.c_uint64), ("n_transient", ctypes.c_uint64),
                ("potential", ctypes.c_int32), ("reserved", ctypes.c_int32)]


def lib():
    """Load liboracle.so, building it first if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            from . import build as _b
            _b.build()
        _lib = load(LIBPATH)
    return _lib


def load(path):
    """Open an oracle shared object at `path` and declare its signatures
    (the tests also load deliberately broken copies this way)."""
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    d, u32, u64, i32 = ctypes.c_double, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    pd = P(d)
    L.oracle_philox.argtypes = [u64, P(u32), P(u32)]
    L.oracle_philox.restype = None
    L.oracle_philox_stream.argtypes = [u64, u32, u32, u32, u64, u64, P(u32)]
    L.oracle_philox_stream.restype = None
    L.oracle_gauss.argtypes = [u64, u32, u32, u32, u64]
    L.oracle_gauss.restype = d
    L.oracle_gauss_stream.argtypes = [u64, u32, u32, u32, u64, u64, pd]
    L.oracle_gauss_stream.restype = None
    L.oracle_jj_integrate.argtypes = [P(JJPoint), u32, P(u32), u64, u64, i32, i32, pd, pd, pd, pd,
                                      u32, pd, pd, i32]
    L.oracle_jj_integrate.restype = i32
    L.oracle_ou_integrate.argtypes = [d, d, d, u64, i32, u64, u32, pd, i32]
    L.oracle_ou_integrate.restype = i32
    L.oracle_kuramoto_integrate.argtypes = [u32, u32, d, d, d, u64, u32, i32, i32, u64, u64,
                                            i32, pd, pd, pd, pd, u32, u32, i32]
    L.oracle_kuramoto_integrate.restype = i32
    L.oracle_kuramoto_rhs.argtypes = [u32, d, i32, pd, pd, pd, pd]
    L.oracle_kuramoto_rhs.restype = None
    return L


def _pd(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def philox(seed, ctr):
    """One Philox4x32-10 block for 64-bit `seed` and 4-word counter `ctr`."""
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    o = (ctypes.c_uint32 * 4)()
    lib().oracle_philox(seed, c, o)
    return [int(x) for x in o]


def philox_stream(seed, tag, a, b, c0_first, count):
    """[count, 4] uint32 array of blocks at counters (c0_first + k, a, b, tag)."""
    out = np.empty((count, 4), dtype=np.uint32)
    lib().oracle_philox_stream(seed, tag, a, b, c0_first, count,
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    return out


def gauss(seed, tag, a, b, n):
    return lib().oracle_gauss(seed, tag, a, b, n)


def gauss_array(seed, tag, a, b, n_first, count):
    """Gaussians n_first .. n_first+count-1 of stream (tag, a, b)."""
    out = np.empty(count, dtype=np.float64)
    lib().oracle_gauss_stream(seed, tag, a, b, n_first, count, _pd(out))
    return out


POT_SIN, POT_SIN2PI = 0, 1


def make_points(params):
    """params: list of dicts with keys m, gamma, a, omega, f, D, n_paths,
    steps_per_period, n_steps, n_transient and optionally potential
    (POT_SIN, the default, or POT_SIN2PI)."""
    arr = (JJPoint * len(params))()
    for i, p in enumerate(params):
        for k, _ in JJPoint._fields_:
            if k == "reserved":
                continue
            setattr(arr[i], k, p.get(k, POT_SIN) if k == "potential" else p[k])
    return arr


def jj_integrate(params, seed, step0=0, scheme=HEUN, state=None, n_record=0, n_threads=0,
                 point_ids=None):
    """Integrate every path of every point.  `state` = (phi, v, acc) float64
    arrays to resume from (copied), else Philox INIT initial conditions.
    `point_ids[q]` replaces q in the Philox counters (a subset of a batch).

    Returns dict(phi, v, acc, point_sums [n_pts,2], rec_phi, rec_v)."""
    pts = make_points(params)
    total = sum(int(p["n_paths"]) for p in params)
    if state is None:
        phi = np.zeros(total); v = np.zeros(total); acc = np.zeros(total)
        init = 0
    else:
        phi, v, acc = (np.array(x, dtype=np.float64, copy=True) for x in state)
        init = 1
    sums = np.zeros((len(params), 2))
    rec_phi = np.zeros((n_record, total)) if n_record else None
    rec_v = np.zeros((n_record, total)) if n_record else None
    ids = None
    if point_ids is not None:
        ids = (ctypes.c_uint32 * len(params))(*[int(x) for x in point_ids])
    rc = lib().oracle_jj_integrate(pts, len(params), ids, seed, step0, scheme, init, _pd(phi),
                                   _pd(v), _pd(acc), _pd(sums), n_record, _pd(rec_phi),
                                   _pd(rec_v), n_threads)
    if rc != 0:
        raise ValueError("oracle_jj_integrate: invalid arguments")
    return dict(phi=phi, v=v, acc=acc, point_sums=sums, rec_phi=rec_phi, rec_v=rec_v)


def ou_integrate(k, D, dt, n_steps, scheme, seed, x0):
    x = np.array(x0, dtype=np.float64, copy=True)
    rc = lib().oracle_ou_integrate(k, D, dt, n_steps, scheme, seed, len(x), _pd(x), 0)
    if rc != 0:
        raise ValueError("oracle_ou_integrate: invalid arguments")
    return x


def kuramoto_integrate(N, R, K, D, dt, n_steps, sample_every, coupling, scheme, seed,
                       omega, Kmat=None, phi0=None, step0=0, r_first=0, r_count=None,
                       n_threads=0):
    """Returns (phi [r_count, N] radians, r_samples [r_count, n_steps//M + 1])."""
    r_count = R - r_first if r_count is None else r_count
    omega = np.ascontiguousarray(omega, dtype=np.float64)
    Km = None if Kmat is None else np.ascontiguousarray(Kmat, dtype=np.float64)
    if phi0 is None:
        phi = np.zeros((r_count, N)); init = 0
    else:
        phi = np.array(phi0, dtype=np.float64, copy=True).reshape(r_count, N); init = 1
    rs = np.zeros((r_count, n_steps // sample_every + 1)) if sample_every else None
    rc = lib().oracle_kuramoto_integrate(N, R, K, D, dt, n_steps, sample_every, coupling,
                                         scheme, seed, step0, init, _pd(phi), _pd(omega),
                                         _pd(Km), _pd(rs), r_first, r_count, n_threads)
    if rc != 0:
        raise ValueError("oracle_kuramoto_integrate: invalid arguments")
    return phi, rs


def kuramoto_rhs(phi, omega, K, coupling, Kmat=None):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    omega = np.ascontiguousarray(omega, dtype=np.float64)
    Km = None if Kmat is None else np.ascontiguousarray(Kmat, dtype=np.float64)
    F = np.zeros_like(phi)
    lib().oracle_kuramoto_rhs(len(phi), K, coupling, _pd(phi), _pd(omega), _pd(Km), _pd(F))
    return F
