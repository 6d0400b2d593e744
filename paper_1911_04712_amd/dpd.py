"""Python binding of the C-ABI in include/dpd.h (argument marshalling only).

Every step of the DPD path runs in the HIP library libdpd.so; this module
allocates the workspace as a torch CUDA tensor, passes torch's current
stream, and converts arrays.  It fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdpd.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENONFINITE, EAGAIN, EBUSY, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6, -7, -8
HOST, DEVICE = 0, 1
POS, VEL, VEL_CENTRED, FORCE = 0, 1, 2, 3
FLAG_VIRIAL = 1
FLAG_REFERENCE_FORCE = 2
FLAG_BODY_UNIFORM = 4
WALL_NONE, WALL_PLATES, WALL_PIPE, WALL_CYLINDERS = 0, 1, 2, 3

_CODES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ESTATE: "ESTATE", ENONFINITE: "ENONFINITE",
          EAGAIN: "EAGAIN", EBUSY: "EBUSY", ENOTFOUND: "ENOTFOUND"}


class DPDError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


class Geom(ctypes.Structure):
    _fields_ = [("cells", ctypes.c_int32 * 3), ("reserved", ctypes.c_int32), ("n", ctypes.c_int64)]


class Params(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("gamma", ctypes.c_double), ("kT", ctypes.c_double),
                ("dt", ctypes.c_double), ("mass", ctypes.c_double), ("body_f", ctypes.c_double),
                ("flow_axis", ctypes.c_int32), ("grad_axis", ctypes.c_int32),
                ("profile_bins", ctypes.c_int32), ("flags", ctypes.c_int32), ("kexp", ctypes.c_double),
                ("wall_kind", ctypes.c_int32), ("reserved2", ctypes.c_int32), ("wall_h", ctypes.c_double),
                ("wall_r_in", ctypes.c_double), ("omega_in", ctypes.c_double), ("omega_out", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("momentum", ctypes.c_double * 3), ("ke_half", ctypes.c_double),
                ("ke_centred", ctypes.c_double), ("kT_centred", ctypes.c_double),
                ("virial", ctypes.c_double), ("pressure", ctypes.c_double),
                ("sum_kT_centred", ctypes.c_double), ("sum_pressure", ctypes.c_double),
                ("sum_momentum", ctypes.c_double * 3), ("nsamples", ctypes.c_uint64),
                ("step", ctypes.c_uint64), ("nonfinite", ctypes.c_int32), ("escaped", ctypes.c_int32)]

    def as_dict(self):
        return {"momentum": np.array(self.momentum), "ke_half": self.ke_half, "ke_centred": self.ke_centred,
                "kT_centred": self.kT_centred, "virial": self.virial, "pressure": self.pressure,
                "sum_kT_centred": self.sum_kT_centred, "sum_pressure": self.sum_pressure,
                "sum_momentum": np.array(self.sum_momentum), "nsamples": int(self.nsamples),
                "step": int(self.step), "nonfinite": int(self.nonfinite), "escaped": int(self.escaped)}


class Request(ctypes.Structure):
    _fields_ = [("geom", Geom), ("params", Params), ("seed", ctypes.c_uint64), ("nsteps", ctypes.c_int64),
                ("pos_n3", ctypes.c_void_p), ("vel_n3", ctypes.c_void_p), ("init_kT", ctypes.c_double),
                ("init_seed", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [("stats", Stats), ("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


# Every symbol include/dpd.h declares, with its ctypes signature.
_VP, _I64 = ctypes.c_void_p, ctypes.c_int64
SIGNATURES = {
    "dpd_position_grid": ([ctypes.POINTER(Geom), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "dpd_workspace_bytes": ([ctypes.POINTER(Geom), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "dpd_create": ([ctypes.POINTER(Geom), _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)], ctypes.c_int),
    "dpd_set_params": ([_VP, ctypes.POINTER(Params)], ctypes.c_int),
    "dpd_set_seed": ([_VP, ctypes.c_uint64], ctypes.c_int),
    "dpd_set_tile": ([_VP, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "dpd_get_tile": ([_VP, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "dpd_set_force_threads": ([_VP, ctypes.c_int32], ctypes.c_int),
    "dpd_get_force_threads": ([_VP, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "dpd_tune_tile": ([_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)],
                      ctypes.c_int),
    "dpd_batch_workspace_bytes": ([ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "dpd_batch_create": ([ctypes.POINTER(_VP), ctypes.c_int32, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)],
                         ctypes.c_int),
    "dpd_batch_step": ([_VP, _I64], ctypes.c_int),
    "dpd_batch_tune": ([_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)],
                       ctypes.c_int),
    "dpd_batch_destroy": ([_VP], ctypes.c_int),
    "dpd_init_random": ([_VP, ctypes.c_double, ctypes.c_uint64], ctypes.c_int),
    "dpd_server_create": ([_VP, ctypes.c_size_t, ctypes.c_int32, _VP, ctypes.POINTER(_VP)], ctypes.c_int),
    "dpd_server_submit": ([_VP, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "dpd_server_pump": ([_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "dpd_server_poll": ([_VP, ctypes.c_uint64, ctypes.POINTER(Result), _VP, _VP], ctypes.c_int),
    "dpd_server_counts": ([_VP, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                           ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "dpd_server_clock": ([_VP], ctypes.c_double),
    "dpd_server_destroy": ([_VP], ctypes.c_int),
    "dpd_set_state": ([_VP, _VP, _VP, ctypes.c_int], ctypes.c_int),
    "dpd_set_step": ([_VP, ctypes.c_uint64], ctypes.c_int),
    "dpd_set_species": ([_VP, ctypes.c_int32, _VP, _VP, _VP], ctypes.c_int),
    "dpd_get_species": ([_VP, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "dpd_set_types": ([_VP, _VP], ctypes.c_int),
    "dpd_set_frozen": ([_VP, _VP], ctypes.c_int),
    "dpd_get_frozen": ([_VP, _VP], ctypes.c_int),
    "dpd_wall_sdf": ([_VP, _VP], ctypes.c_int),
    "dpd_get_types": ([_VP, _VP], ctypes.c_int),
    "dpd_build_cells": ([_VP], ctypes.c_int),
    "dpd_step": ([_VP, _I64], ctypes.c_int),
    "dpd_prepare_steps": ([_VP, _I64], ctypes.c_int),
    "dpd_time_force": ([_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "dpd_read": ([_VP, ctypes.c_int, _VP, ctypes.c_int], ctypes.c_int),
    "dpd_read_raw": ([_VP, _VP, _VP, _VP, ctypes.c_int], ctypes.c_int),
    "dpd_get_stats": ([_VP, ctypes.POINTER(Stats)], ctypes.c_int),
    "dpd_get_profile": ([_VP, _VP, _VP, ctypes.c_int32], ctypes.c_int),
    "dpd_reset_accumulators": ([_VP], ctypes.c_int),
    "dpd_destroy": ([_VP], ctypes.c_int),
    "dpd_profile_steps": ([_VP, _I64, _VP], ctypes.c_int),
    "dpd_last_error": ([], ctypes.c_char_p),
    "dpd_set_tune_cache": ([ctypes.c_char_p], ctypes.c_int),
    "dpd_philox": ([_VP, _VP, _I64, _VP, ctypes.c_int, _VP], ctypes.c_int),
    "dpd_box_muller": ([_VP, _VP, _I64, _VP, ctypes.c_int, _VP], ctypes.c_int),
    "dpd_run_static": ([ctypes.POINTER(Geom), ctypes.POINTER(Params), ctypes.c_uint64, ctypes.c_uint64, _VP, _VP,
                        _I64, _VP, _VP, ctypes.POINTER(Stats), _VP], ctypes.c_int),
}

# Bytes of the library's static per-GPU machine array (DPD_STATIC_WS_BYTES).
STATIC_WS_BYTES = 64 * 1024 * 1024

_lib = None


def lib():
    """Load libdpd.so (never builds; build with paper_1911_04712_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1911_04712_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise DPDError(rc, lib().dpd_last_error().decode(errors="replace"))
    return rc


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the DPD library needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _stream_ptr(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def set_tune_cache(path):
    """Use (or with None stop using) a JSON autotuner cache file: tuners
    apply stored tiles without timing and add what they time."""
    _check(lib().dpd_set_tune_cache(None if path is None else os.fsencode(path)))


def make_geom(cells, n):
    return Geom((ctypes.c_int32 * 3)(*[int(c) for c in cells]), 0, int(n))


def position_grid(cells, n=0):
    q = ctypes.c_double()
    _check(lib().dpd_position_grid(ctypes.byref(make_geom(cells, n)), ctypes.byref(q)))
    return q.value


def workspace_bytes(cells, n):
    b = ctypes.c_size_t()
    _check(lib().dpd_workspace_bytes(ctypes.byref(make_geom(cells, n)), ctypes.byref(b)))
    return b.value


def batch_workspace_bytes(nboxes):
    b = ctypes.c_size_t()
    _check(lib().dpd_batch_workspace_bytes(int(nboxes), ctypes.byref(b)))
    return b.value


def make_params(a=25.0, gamma=4.5, kT=1.0, dt=0.01, mass=1.0, body_f=0.0, flow_axis=0, grad_axis=1,
                profile_bins=0, flags=0, kexp=1.0, wall_kind=0, wall_h=0.0, wall_r_in=0.0, omega_in=0.0,
                omega_out=0.0):
    """kexp: exponent k of the random-term kernel w_R = (1 - r)^k (0 < k <= 1).
    wall_kind: WALL_NONE, WALL_PLATES (half-gap wall_h), WALL_PIPE (radius
    wall_h) or WALL_CYLINDERS (radii wall_r_in < wall_h, turning at omega_in
    and omega_out about +flow_axis)."""
    return Params(float(a), float(gamma), float(kT), float(dt), float(mass), float(body_f), int(flow_axis),
                  int(grad_axis), int(profile_bins), int(flags), float(kexp), int(wall_kind), 0, float(wall_h),
                  float(wall_r_in), float(omega_in), float(omega_out))


def _as_arg(arr, dtype, shape_tail):
    """(pointer, where, keepalive) for a numpy array or a torch CUDA tensor."""
    try:
        import torch
        if isinstance(arr, torch.Tensor):
            if not arr.is_cuda:
                arr = arr.numpy()
            else:
                t = arr.contiguous()
                return ctypes.c_void_p(t.data_ptr()), DEVICE, t
    except ImportError:
        pass
    a = np.ascontiguousarray(arr, dtype=dtype)
    if shape_tail is not None:
        a = a.reshape(-1, shape_tail)
    return a.ctypes.data_as(ctypes.c_void_p), HOST, a


class Box:
    """One periodic DPD box resident in a torch-allocated HBM workspace."""

    def __init__(self, cells, n, params=None, seed=None, device="cuda"):
        torch = _torch()
        self.cells = tuple(int(c) for c in cells)
        self.n = int(n)
        self.ws_bytes = workspace_bytes(self.cells, self.n)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self._h = ctypes.c_void_p()
        _check(lib().dpd_create(ctypes.byref(make_geom(self.cells, self.n)), ctypes.c_void_p(self.ws.data_ptr()),
                                self.ws_bytes, _stream_ptr(torch), ctypes.byref(self._h)))
        self.params = None
        if params is not None:
            self.set_params(params)
        if seed is not None:
            self.set_seed(seed)

    # -- setup --------------------------------------------------------------
    def set_params(self, params=None, **kw):
        p = params if isinstance(params, Params) else make_params(**(params or {}), **kw)
        _check(lib().dpd_set_params(self._h, ctypes.byref(p)))
        self.params = p

    def set_tile(self, tile):
        t = (ctypes.c_int32 * 3)(*[int(x) for x in tile])
        _check(lib().dpd_set_tile(self._h, t))

    def get_tile(self):
        t = (ctypes.c_int32 * 3)()
        _check(lib().dpd_get_tile(self._h, t))
        return tuple(t)

    def set_force_threads(self, threads):
        """Workgroup size of the tile force kernel: 256, 512, 1024 (0: default)."""
        _check(lib().dpd_set_force_threads(self._h, int(threads)))

    def get_force_threads(self):
        t = ctypes.c_int32()
        _check(lib().dpd_get_force_threads(self._h, ctypes.byref(t)))
        return t.value

    def tune_tile(self, reps=5):
        """Time the force kernel for the candidate tiles and keep the fastest.
        Returns (tile, ms per force evaluation)."""
        t = (ctypes.c_int32 * 3)()
        ms = ctypes.c_double()
        _check(lib().dpd_tune_tile(self._h, int(reps), t, ctypes.byref(ms)))
        return tuple(t), ms.value

    def set_seed(self, seed):
        _check(lib().dpd_set_seed(self._h, int(seed) & 0xFFFFFFFFFFFFFFFF))

    def set_state(self, pos, vel):
        pp, wp, k1 = _as_arg(pos, np.float32, 3)
        vp, wv, k2 = _as_arg(vel, np.float32, 3)
        if wp != wv:
            raise ValueError("pos and vel must both be host arrays or both device tensors")
        _check(lib().dpd_set_state(self._h, pp, vp, wp))

    def set_step(self, step):
        """Index of the next force evaluation (resuming a run)."""
        _check(lib().dpd_set_step(self._h, int(step)))

    def set_species(self, a_tab=None, gamma_tab=None, rc_tab=None):
        """Per species-pair a, gamma and cutoff (symmetric ntypes x ntypes
        tables; no rc_tab: every cutoff 1); no tables returns to the single
        species of the params."""
        if a_tab is None:
            _check(lib().dpd_set_species(self._h, 0, None, None, None))
            return
        a = np.ascontiguousarray(a_tab, dtype=np.float64)
        g = np.ascontiguousarray(gamma_tab, dtype=np.float64)
        if a.ndim != 2 or a.shape[0] != a.shape[1] or g.shape != a.shape:
            raise ValueError("a_tab and gamma_tab must be square tables of one shape")
        c = None if rc_tab is None else np.ascontiguousarray(rc_tab, dtype=np.float64)
        if c is not None and c.shape != a.shape:
            raise ValueError("rc_tab must have the shape of a_tab")
        _check(lib().dpd_set_species(self._h, a.shape[0], a.ctypes.data, g.ctypes.data,
                                     None if c is None else c.ctypes.data))

    def get_species(self):
        nt = ctypes.c_int32()
        _check(lib().dpd_get_species(self._h, ctypes.byref(nt)))
        return nt.value

    def set_types(self, types):
        """Species of particle id i = types[i] (host array of n ints)."""
        t = np.ascontiguousarray(types, dtype=np.int32)
        if t.shape != (self.n,):
            raise ValueError(f"types must have shape ({self.n},)")
        _check(lib().dpd_set_types(self._h, t.ctypes.data))

    def get_types(self):
        t = np.empty(self.n, dtype=np.int32)
        _check(lib().dpd_get_types(self._h, t.ctypes.data))
        return t

    def set_frozen(self, frozen):
        """Mark wall particles: frozen[i] true freezes particle id i."""
        f = np.ascontiguousarray(np.asarray(frozen).astype(bool), dtype=np.uint8)
        if f.shape != (self.n,):
            raise ValueError(f"frozen must have shape ({self.n},)")
        _check(lib().dpd_set_frozen(self._h, f.ctypes.data))

    def get_frozen(self):
        f = np.empty(self.n, dtype=np.uint8)
        _check(lib().dpd_get_frozen(self._h, f.ctypes.data))
        return f.astype(bool)

    def wall_sdf(self):
        """Signed wall distance of every particle (id order; negative in the fluid)."""
        out = np.empty(self.n, dtype=np.float32)
        _check(lib().dpd_wall_sdf(self._h, out.ctypes.data))
        return out

    def init_random(self, kT, seed):
        """Random state generated on the device (uniform positions, Maxwellian
        velocities with the centre-of-mass velocity removed)."""
        _check(lib().dpd_init_random(self._h, float(kT), int(seed) & 0xFFFFFFFFFFFFFFFF))

    # -- stepping -----------------------------------------------------------
    def build_cells(self):
        _check(lib().dpd_build_cells(self._h))

    def step(self, nsteps=1):
        _check(lib().dpd_step(self._h, int(nsteps)))

    def prepare(self, nsteps):
        """Capture the graphs a step(nsteps) would launch (nothing runs)."""
        _check(lib().dpd_prepare_steps(self._h, int(nsteps)))

    def time_force(self, reps=20):
        """Mean ms per launch of the pair-force kernel alone on the current
        positions (the state does not advance)."""
        ms = ctypes.c_double()
        _check(lib().dpd_time_force(self._h, int(reps), ctypes.byref(ms)))
        return ms.value

    def profile_steps(self, nsteps):
        """Mean device ms per step of each stage (bin, force, virial, integrate)
        of eager steps, timed by events that each stage's first kernel records
        as it starts and its last as it ends."""
        ms = np.zeros(4)
        _check(lib().dpd_profile_steps(self._h, int(nsteps), ms.ctypes.data_as(ctypes.c_void_p)))
        return dict(zip(("bin", "force", "virial", "integrate"), ms.tolist()))

    # -- reads --------------------------------------------------------------
    def read(self, what=POS, out=None):
        """n x 3 float32 rows in id order (numpy, or into a CUDA tensor `out`)."""
        if out is not None:
            op, w, keep = _as_arg(out, np.float32, None)
            _check(lib().dpd_read(self._h, int(what), op, w))
            return out
        a = np.empty((self.n, 3), dtype=np.float32)
        _check(lib().dpd_read(self._h, int(what), a.ctypes.data_as(ctypes.c_void_p), HOST))
        return a

    def read_raw(self):
        """(pos4, vel4, cell_start) of the last binning, in cell order."""
        nc = self.cells[0] * self.cells[1] * self.cells[2]
        p4 = np.empty((self.n, 4), dtype=np.float32)
        v4 = np.empty((self.n, 4), dtype=np.float32)
        cs = np.empty(nc + 1, dtype=np.int32)
        _check(lib().dpd_read_raw(self._h, p4.ctypes.data_as(ctypes.c_void_p), v4.ctypes.data_as(ctypes.c_void_p),
                                  cs.ctypes.data_as(ctypes.c_void_p), HOST))
        return p4, v4, cs

    def stats(self, allow_nonfinite=False):
        s = Stats()
        rc = lib().dpd_get_stats(self._h, ctypes.byref(s))
        if rc != OK and not (allow_nonfinite and rc == ENONFINITE):
            _check(rc)
        return s.as_dict()

    def profile(self):
        nb = int(self.params.profile_bins)
        sv = np.zeros(nb)
        cn = np.zeros(nb)
        _check(lib().dpd_get_profile(self._h, sv.ctypes.data_as(ctypes.c_void_p), cn.ctypes.data_as(ctypes.c_void_p),
                                     nb))
        return sv, cn

    def reset_accumulators(self):
        _check(lib().dpd_reset_accumulators(self._h))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().dpd_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Many boxes stepped together: one launch per kernel for all boxes, one
    captured graph for a whole run."""

    def __init__(self, boxes):
        torch = _torch()
        self.boxes = list(boxes)
        nb = len(self.boxes)
        b = ctypes.c_size_t()
        _check(lib().dpd_batch_workspace_bytes(nb, ctypes.byref(b)))
        self.ws = torch.empty(b.value, dtype=torch.uint8, device="cuda")
        arr = (_VP * nb)(*[bx._h.value for bx in self.boxes])
        self._h = ctypes.c_void_p()
        _check(lib().dpd_batch_create(arr, nb, ctypes.c_void_p(self.ws.data_ptr()), b.value, _stream_ptr(torch),
                                      ctypes.byref(self._h)))

    def step(self, nsteps):
        _check(lib().dpd_batch_step(self._h, int(nsteps)))

    def tune(self, reps=5):
        """Batch autotuner: returns (uniform tile or None when the boxes'
        own tiles were fastest, ms per batched force evaluation)."""
        t = (ctypes.c_int32 * 3)()
        ms = ctypes.c_double()
        _check(lib().dpd_batch_tune(self._h, int(reps), t, ctypes.byref(ms)))
        return (tuple(t) if t[0] > 0 else None), ms.value

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().dpd_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request server over one torch-allocated HBM pool."""

    def __init__(self, pool_bytes, max_slots=256):
        torch = _torch()
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device="cuda")
        self._h = ctypes.c_void_p()
        _check(lib().dpd_server_create(ctypes.c_void_p(self.pool.data_ptr()), int(pool_bytes), int(max_slots),
                                       _stream_ptr(torch), ctypes.byref(self._h)))
        self._sizes = {}

    def submit(self, cells, n, params, seed, nsteps, pos=None, vel=None, init_kT=1.0, init_seed=0):
        keep = []
        pp = vp = None
        if pos is not None:
            pa = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)
            va = np.ascontiguousarray(vel, dtype=np.float32).reshape(-1, 3)
            keep += [pa, va]
            pp, vp = pa.ctypes.data_as(ctypes.c_void_p), va.ctypes.data_as(ctypes.c_void_p)
        p = params if isinstance(params, Params) else make_params(**params)
        r = Request(make_geom(cells, n), p, int(seed) & 0xFFFFFFFFFFFFFFFF, int(nsteps), pp, vp, float(init_kT),
                    int(init_seed) & 0xFFFFFFFFFFFFFFFF)
        t = ctypes.c_uint64()
        _check(lib().dpd_server_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        self._sizes[t.value] = int(n)
        return t.value

    def pump(self, quantum):
        ran = ctypes.c_int32()
        _check(lib().dpd_server_pump(self._h, int(quantum), ctypes.byref(ran)))
        return ran.value

    def poll(self, ticket, want_state=False):
        """None while running; then (result dict, pos, vel) once (pos/vel None
        unless want_state)."""
        res = Result()
        n = self._sizes.get(ticket, 0)
        pos = vel = None
        pp = vp = None
        if want_state:
            pos = np.empty((n, 3), dtype=np.float32)
            vel = np.empty((n, 3), dtype=np.float32)
            pp, vp = pos.ctypes.data_as(ctypes.c_void_p), vel.ctypes.data_as(ctypes.c_void_p)
        rc = lib().dpd_server_poll(self._h, int(ticket), ctypes.byref(res), pp, vp)
        if rc == EAGAIN:
            return None
        _check(rc)
        self._sizes.pop(ticket, None)
        out = {"status": res.status, "t_submit": res.t_submit, "t_admit": res.t_admit, "t_done": res.t_done,
               "stats": res.stats.as_dict()}
        return out, pos, vel

    def counts(self):
        q, a, ps = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib().dpd_server_counts(self._h, ctypes.byref(q), ctypes.byref(a), ctypes.byref(ps)))
        return q.value, a.value, ps.value

    def clock(self):
        return lib().dpd_server_clock(self._h)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().dpd_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_static(cells, pos, vel, params, seed, nsteps, step0=0, pos_out=None, vel_out=None, allow_nonfinite=False):
    """One whole run in the library's static per-GPU machine array
    (dpd_run_static: no device allocation by the library).  pos, vel: torch
    CUDA float32 tensors (n, 3), row = id (numpy arrays are copied to the
    GPU first); pos_out, vel_out: torch CUDA float32 (n, 3) tensors, made if
    None.  Returns (pos_out, vel_out, stats)."""
    torch = _torch()

    def dev(a):
        if isinstance(a, torch.Tensor) and a.is_cuda:
            return a.to(torch.float32).contiguous()
        return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32).reshape(-1, 3), device="cuda")

    p, v = dev(pos), dev(vel)
    n = p.shape[0]
    po = torch.empty((n, 3), dtype=torch.float32, device="cuda") if pos_out is None else pos_out
    vo = torch.empty((n, 3), dtype=torch.float32, device="cuda") if vel_out is None else vel_out
    for t in (po, vo):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and tuple(t.shape) == (n, 3)):
            raise ValueError("pos_out / vel_out must be contiguous CUDA float32 tensors of shape (n, 3)")
    st = Stats()
    prm = params if params is not None else make_params()
    rc = lib().dpd_run_static(ctypes.byref(make_geom(cells, n)), ctypes.byref(prm), int(seed) & 0xFFFFFFFFFFFFFFFF,
                              int(step0), ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(v.data_ptr()), int(nsteps),
                              ctypes.c_void_p(po.data_ptr()), ctypes.c_void_p(vo.data_ptr()), ctypes.byref(st),
                              _stream_ptr(torch))
    if not (allow_nonfinite and rc == ENONFINITE):
        _check(rc)
    return po, vo, st.as_dict()


def philox(ctr4, key2):
    """Philox4x32-10 words computed on the GPU (uint32 arrays n x 4, n x 2)."""
    torch = _torch()
    c = torch.as_tensor(np.ascontiguousarray(ctr4, dtype=np.uint32).view(np.int32), device="cuda")
    k = torch.as_tensor(np.ascontiguousarray(key2, dtype=np.uint32).view(np.int32), device="cuda")
    n = c.shape[0]
    out = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    _check(lib().dpd_philox(ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(k.data_ptr()), n,
                            ctypes.c_void_p(out.data_ptr()), DEVICE, _stream_ptr(torch)))
    return out.cpu().numpy().view(np.uint32)


def box_muller(w0, w1):
    """FP32 Box-Muller of the force kernel, on the GPU."""
    torch = _torch()
    a = torch.as_tensor(np.ascontiguousarray(w0, dtype=np.uint32).view(np.int32), device="cuda")
    b = torch.as_tensor(np.ascontiguousarray(w1, dtype=np.uint32).view(np.int32), device="cuda")
    out = torch.empty(a.shape[0], dtype=torch.float32, device="cuda")
    _check(lib().dpd_box_muller(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), a.shape[0],
                                ctypes.c_void_p(out.data_ptr()), DEVICE, _stream_ptr(torch)))
    return out.cpu().numpy()
