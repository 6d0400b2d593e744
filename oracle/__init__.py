"""ctypes wrapper of the CPU oracle (oracle/orc.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the GPU library.  Plain FP64;
see orc.c for the passages of the paper each function follows.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# DPD_ORACLE_SANITIZED=1 selects the ASan/UBSan build (see oracle/build.py)
_SANITIZED = os.environ.get("DPD_ORACLE_SANITIZED", "") == "1"
_LIB_PATH = os.path.join(_HERE, "liborc_san.so" if _SANITIZED else "liborc.so")
_lib = None


class Params(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("gamma", ctypes.c_double), ("kT", ctypes.c_double),
                ("dt", ctypes.c_double), ("mass", ctypes.c_double), ("body_f", ctypes.c_double),
                ("flow_axis", ctypes.c_int32), ("grad_axis", ctypes.c_int32), ("kexp", ctypes.c_double),
                ("ntypes", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("type", ctypes.POINTER(ctypes.c_int32)), ("a_tab", ctypes.POINTER(ctypes.c_double)),
                ("g_tab", ctypes.POINTER(ctypes.c_double)),
                ("body_uniform", ctypes.c_int32), ("wall_kind", ctypes.c_int32), ("wall_h", ctypes.c_double),
                ("frozen", ctypes.POINTER(ctypes.c_uint8)), ("rc", ctypes.c_double),
                ("rc_tab", ctypes.POINTER(ctypes.c_double)), ("wall_r_in", ctypes.c_double),
                ("omega_in", ctypes.c_double), ("omega_out", ctypes.c_double)]


class Diag(ctypes.Structure):
    _fields_ = [("momentum", ctypes.c_double * 3), ("ke_half", ctypes.c_double),
                ("ke_centred", ctypes.c_double), ("kT_centred", ctypes.c_double),
                ("virial", ctypes.c_double), ("pressure", ctypes.c_double)]


def _p(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build
            build.build(sanitize=_SANITIZED)
        L = ctypes.CDLL(_LIB_PATH)
        u32p, u64p, i64p, i32p = (ctypes.POINTER(t) for t in
                                  (ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32))
        dp, fp = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_philox_batch.argtypes = [ctypes.c_int64, u32p, u32p, u32p]
        L.orc_box_muller.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.orc_box_muller.restype = ctypes.c_double
        L.orc_box_muller_batch.argtypes = [ctypes.c_int64, u32p, u32p, dp]
        L.orc_pair_words.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, u32p]
        L.orc_xi.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64]
        L.orc_xi.restype = ctypes.c_double
        L.orc_xi_batch.argtypes = [ctypes.c_int64, u32p, u32p, u64p, ctypes.c_uint64, dp]
        L.orc_bin.argtypes = [ctypes.c_int64, fp, i32p, i64p, i32p]
        L.orc_pair_force.argtypes = [dp, dp, dp, dp, dp, ctypes.POINTER(Params), ctypes.c_uint32,
                                     ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, dp, dp, dp]
        L.orc_forces.argtypes = [ctypes.c_int64, dp, dp, u32p, i32p, ctypes.POINTER(Params),
                                 ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_int64, i64p,
                                 dp, dp, dp]
        L.orc_step.argtypes = [ctypes.c_int64, dp, dp, u32p, i32p, ctypes.POINTER(Params),
                               ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32,
                               ctypes.POINTER(Diag), dp, dp, dp]
        L.orc_sdf.argtypes = [dp, i32p, ctypes.POINTER(Params)]
        L.orc_sdf.restype = ctypes.c_double
        L.orc_wall_velocity.argtypes = [dp, i32p, ctypes.POINTER(Params), dp]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def make_params(a=25.0, gamma=4.5, kT=1.0, dt=0.01, mass=1.0, body_f=0.0, flow_axis=0, grad_axis=1, kexp=1.0):
    """kexp: exponent k of the random-term kernel w_R = (1 - r)^k (0 < k <= 1)."""
    return Params(float(a), float(gamma), float(kT), float(dt), float(mass), float(body_f),
                  int(flow_axis), int(grad_axis), float(kexp))


def with_species(params, types, a_tab, g_tab, rc_tab=None):
    """Copy of params for a mixture: types[i] is the species of row i of the
    state, a_tab / g_tab (/ rc_tab) the symmetric ntypes x ntypes tables of
    a, gamma (and the cutoff, <= 1) per species pair.  The arrays are kept
    alive by the returned object."""
    t = np.ascontiguousarray(types, dtype=np.int32)
    a = np.ascontiguousarray(a_tab, dtype=np.float64)
    g = np.ascontiguousarray(g_tab, dtype=np.float64)
    nt = a.shape[0]
    assert a.shape == (nt, nt) and g.shape == (nt, nt)
    q = Params()
    ctypes.pointer(q)[0] = params
    q.ntypes, q.type, q.a_tab, q.g_tab = nt, _p(t, ctypes.c_int32), _p(a, ctypes.c_double), _p(g, ctypes.c_double)
    keep = [t, a, g]
    if rc_tab is not None:
        c = np.ascontiguousarray(rc_tab, dtype=np.float64)
        assert c.shape == (nt, nt)
        q.rc_tab = _p(c, ctypes.c_double)
        keep.append(c)
    q._keep = tuple(keep)
    return q


def with_walls(params, kind, h, frozen=None, body_uniform=True, r_in=0.0, omega_in=0.0, omega_out=0.0):
    """Copy of params with walls: kind 1 = two plates normal to grad_axis
    (fluid where |y - L/2| < h), 2 = a pipe of radius h along flow_axis
    through the box centre, 3 = coaxial cylinders of radii r_in < h along
    flow_axis turning at omega_in and omega_out; frozen[i] = 1 marks a wall
    particle.  The body force becomes uniform unless body_uniform is False."""
    q = Params()
    ctypes.pointer(q)[0] = params
    keep = list(getattr(params, "_keep", ()))
    q.wall_kind, q.wall_h, q.body_uniform = int(kind), float(h), int(bool(body_uniform))
    q.wall_r_in, q.omega_in, q.omega_out = float(r_in), float(omega_in), float(omega_out)
    if frozen is not None:
        fz = np.ascontiguousarray(frozen, dtype=np.uint8)
        q.frozen = _p(fz, ctypes.c_uint8)
        keep.append(fz)
    q._keep = tuple(keep)
    return q


def sdf(points, cells, params):
    """The oracle's signed wall distance at each point (negative in the fluid)."""
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    c = np.ascontiguousarray(cells, dtype=np.int32)
    L = lib()
    return np.array([L.orc_sdf(_p(pts[k], ctypes.c_double), _p(c, ctypes.c_int32), ctypes.byref(params))
                     for k in range(len(pts))])


def wall_velocity(points, cells, params):
    """The oracle's wall velocity field at each point."""
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    c = np.ascontiguousarray(cells, dtype=np.int32)
    out = np.zeros_like(pts)
    L = lib()
    for k in range(len(pts)):
        L.orc_wall_velocity(_p(pts[k], ctypes.c_double), _p(c, ctypes.c_int32), ctypes.byref(params),
                            _p(out[k], ctypes.c_double))
    return out


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(key, dtype=np.uint32).reshape(2)
    out = np.empty_like(c)
    lib().orc_philox_batch(len(c), _p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32), _p(out, ctypes.c_uint32))
    return out


def pair_words(id_a, id_b, step, seed):
    out = np.empty(4, dtype=np.uint32)
    lib().orc_pair_words(id_a, id_b, step, seed, _p(out, ctypes.c_uint32))
    return out


def box_muller(w0, w1):
    return lib().orc_box_muller(int(w0), int(w1))


def box_muller_batch(w0, w1):
    a = np.ascontiguousarray(w0, dtype=np.uint32)
    b = np.ascontiguousarray(w1, dtype=np.uint32)
    out = np.empty(a.shape, dtype=np.float64)
    lib().orc_box_muller_batch(a.size, _p(a, ctypes.c_uint32), _p(b, ctypes.c_uint32), _p(out, ctypes.c_double))
    return out


def xi(id_a, id_b, step, seed):
    return lib().orc_xi(int(id_a), int(id_b), int(step), int(seed))


def xi_batch(id_a, id_b, step, seed):
    a = np.ascontiguousarray(id_a, dtype=np.uint32)
    b = np.ascontiguousarray(id_b, dtype=np.uint32)
    s = np.ascontiguousarray(np.broadcast_to(np.asarray(step, dtype=np.uint64), a.shape))
    out = np.empty(a.shape, dtype=np.float64)
    lib().orc_xi_batch(a.size, _p(a, ctypes.c_uint32), _p(b, ctypes.c_uint32), _p(s, ctypes.c_uint64),
                       int(seed), _p(out, ctypes.c_double))
    return out


def bin_cells(pos3_f32, cells):
    """Stable counting sort of FP32 positions into unit cells.
    Returns (order, cell_start): order[k] = input index of the k-th particle."""
    pos = np.ascontiguousarray(pos3_f32, dtype=np.float32).reshape(-1, 3)
    c = np.ascontiguousarray(cells, dtype=np.int32)
    nc = int(c[0]) * int(c[1]) * int(c[2])
    order = np.empty(len(pos), dtype=np.int64)
    start = np.empty(nc + 1, dtype=np.int32)
    rc = lib().orc_bin(len(pos), _p(pos, ctypes.c_float), _p(c, ctypes.c_int32), _p(order, ctypes.c_int64),
                       _p(start, ctypes.c_int32))
    if rc:
        raise RuntimeError(f"orc_bin failed ({rc})")
    return order, start


def pair_force(ri, rj, vi, vj, box, params, id_i=0, id_j=1, step=0, seed=0):
    """Force on i from j (total, conservative part, error scale)."""
    args = [np.ascontiguousarray(a, dtype=np.float64) for a in (ri, rj, vi, vj, box)]
    F, Fc, mag = np.zeros(3), np.zeros(3), np.zeros(1)
    hit = lib().orc_pair_force(*(_p(a, ctypes.c_double) for a in args), ctypes.byref(params),
                               int(id_i), int(id_j), int(step), int(seed), _p(F, ctypes.c_double),
                               _p(Fc, ctypes.c_double), _p(mag, ctypes.c_double))
    return bool(hit), F, Fc, float(mag[0])


def forces(x, v, ids, cells, params, step, seed, brute=False, which=None):
    """Forces f (pair sum + body force), error scale s and the conservative
    virial at one instant.  `which` limits evaluation to a subset."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, 3)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    c = np.ascontiguousarray(cells, dtype=np.int32)
    n = len(x)
    if which is None:
        m, wp, cnt = 0, None, n
    else:
        w = np.ascontiguousarray(which, dtype=np.int64)
        m, wp, cnt = len(w), _p(w, ctypes.c_int64), len(w)
    f = np.zeros((cnt, 3))
    s = np.zeros(cnt)
    vir = np.zeros(1)
    rc = lib().orc_forces(n, _p(x, ctypes.c_double), _p(v, ctypes.c_double), _p(ids, ctypes.c_uint32),
                          _p(c, ctypes.c_int32), ctypes.byref(params), int(step), int(seed), int(bool(brute)),
                          m, wp, _p(f, ctypes.c_double), _p(s, ctypes.c_double), _p(vir, ctypes.c_double))
    if rc:
        raise RuntimeError(f"orc_forces failed ({rc})")
    return f, s, float(vir[0])


def step(x, v, ids, cells, params, seed, step0, nsteps, nbins=0, want_diag=True):
    """Advance (x, v) in place by nsteps.  Returns (diag records, profile
    sums, profile counts, forces of the last step)."""
    assert x.dtype == np.float64 and x.flags.c_contiguous
    assert v.dtype == np.float64 and v.flags.c_contiguous
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    c = np.ascontiguousarray(cells, dtype=np.int32)
    n = len(x)
    diag = (Diag * max(int(nsteps), 1))() if want_diag else None
    ps = np.zeros(max(nbins, 1))
    pc = np.zeros(max(nbins, 1))
    fl = np.zeros((n, 3))
    rc = lib().orc_step(n, _p(x, ctypes.c_double), _p(v, ctypes.c_double), _p(ids, ctypes.c_uint32),
                        _p(c, ctypes.c_int32), ctypes.byref(params), int(seed), int(step0), int(nsteps),
                        int(nbins), diag, _p(ps, ctypes.c_double), _p(pc, ctypes.c_double),
                        _p(fl, ctypes.c_double))
    if rc:
        raise RuntimeError(f"orc_step failed ({rc})")
    recs = None
    if want_diag:
        recs = {
            "momentum": np.array([list(d.momentum) for d in diag[:nsteps]]),
            "ke_half": np.array([d.ke_half for d in diag[:nsteps]]),
            "ke_centred": np.array([d.ke_centred for d in diag[:nsteps]]),
            "kT_centred": np.array([d.kT_centred for d in diag[:nsteps]]),
            "virial": np.array([d.virial for d in diag[:nsteps]]),
            "pressure": np.array([d.pressure for d in diag[:nsteps]]),
        }
    return recs, ps[:nbins], pc[:nbins], fl


def num_threads():
    return int(lib().orc_num_threads())


def set_num_threads(t):
    lib().orc_set_num_threads(int(t))
