"""Thin ctypes binding of ``libsusp.so`` (C ABI in ``include/susp.h``).

Only argument marshalling lives here: every part of the step runs in the HIP library.
PyTorch provides the device memory (a workspace tensor) and the HIP stream.  Importing
this module on a machine without the built library raises; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsusp.so")

FP64, FP32, FP16STORE = 0, 1, 2
LIST_OWNER, LIST_GHOST, LIST_CELLS, LIST_PAIRS, LIST_CONTACTS, LIST_LINKS = range(6)
OK, EINVAL, ENOMEM, EDEVICE, EUNSTABLE, ESTATE = 0, -1, -2, -3, -4, -5

_PD = C.POINTER(C.c_double)
_PI = C.POINTER(C.c_int32)


class Params(C.Structure):
    _fields_ = [
        ("lx", C.c_int32), ("ly", C.c_int32), ("lz", C.c_int32), ("precision", C.c_int32),
        ("tau", C.c_double), ("rho0", C.c_double),
        ("n", C.c_int32), ("pos", _PD), ("vel", _PD), ("omega", _PD), ("radius", _PD),
        ("map_ratio", C.c_double), ("rho_p", C.c_double),
        ("kn", C.c_double), ("kt_ratio", C.c_double), ("mu", C.c_double), ("eta_n", C.c_double),
        ("lub_delta", C.c_double), ("lub_hc", C.c_double), ("lub_subtract_hc", C.c_int32),
        ("F0", C.c_double), ("debye_lambda", C.c_double), ("pair_cutoff", C.c_double),
        ("n_sub", C.c_int32), ("quasi2d", C.c_int32),
        ("shear_kind", C.c_int32), ("gamma_dot", C.c_double), ("g0_I", C.c_double),
        ("g0_F", C.c_double), ("period", C.c_int32), ("theta", C.c_double),
        ("ncyc_I", C.c_int32), ("ncyc_F", C.c_int32), ("fp16_exp", C.c_int32),
        ("brick_y", C.c_int32), ("brick_z", C.c_int32), ("contact_bins", C.c_int32),
        ("collision", C.c_int32), ("tau_bulk", C.c_double), ("tau_ghost", C.c_double),
        ("lub_implicit", C.c_int32), ("boundary", C.c_int32), ("wall", _PI),
    ]


class SuspError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("susp error %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsusp.so is not built (run __graft_entry__.build() or "
                              "python paper_1904_02929_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.susp_default_params.argtypes = [C.POINTER(Params)]
        L.susp_footprint_bytes.argtypes = [C.POINTER(Params)]
        L.susp_footprint_bytes.restype = C.c_size_t
        L.susp_create.argtypes = [C.POINTER(Params), vp, vp, C.c_size_t, C.POINTER(vp)]
        L.susp_step.argtypes = [vp, C.c_int64]
        L.susp_stress.argtypes = [vp, _PD, _PD]
        L.susp_contact_stats.argtypes = [vp, C.c_int32, _PD, _PD]
        L.susp_contact_stats_noalloc.argtypes = [vp, C.c_int32, _PD, _PD]
        L.susp_wall_force.argtypes = [vp, _PD]
        L.susp_destroy.argtypes = [vp]
        L.susp_get_populations.argtypes = [vp, _PD]
        L.susp_set_populations.argtypes = [vp, _PD]
        L.susp_get_particles.argtypes = [vp, _PD, _PD, _PD, _PD]
        L.susp_set_particles.argtypes = [vp, _PD, _PD, _PD, _PD]
        L.susp_get_history.argtypes = [vp, C.c_int32, _PI, _PI, _PI, _PD]
        L.susp_set_history.argtypes = [vp, C.c_int32, _PI, _PI, _PD]
        L.susp_get_clock.argtypes = [vp, C.POINTER(C.c_int64), _PD]
        L.susp_set_clock.argtypes = [vp, C.c_int64]
        L.susp_get_hydro.argtypes = [vp, _PD, _PD, _PD, _PI]
        L.susp_get_lists.argtypes = [vp, C.c_int32, vp, C.POINTER(C.c_size_t)]
        L.susp_get_derived.argtypes = [vp, _PD]
        L.susp_get_accumulators.argtypes = [vp, _PD]
        L.susp_profile_read_parts.argtypes = [vp, _PD, C.POINTER(C.c_int64)]
        L.susp_health.argtypes = [vp, _PD]
        L.susp_set_accumulators.argtypes = [vp, _PD]
        L.susp_get_state.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
        L.susp_set_state.argtypes = [vp, vp, C.c_size_t]
        L.susp_use_graphs.argtypes = [vp, C.c_int32]
        L.susp_profile.argtypes = [vp, C.c_int32]
        L.susp_profile_read.argtypes = [vp, _PD, C.POINTER(C.c_int64)]
        L.susp_last_error.restype = C.c_char_p
        L.susp_batch_create.argtypes = [C.c_int32, C.c_size_t, C.c_int32, C.POINTER(vp)]
        L.susp_batch_add.argtypes = [vp, C.POINTER(Params), C.POINTER(C.c_int32)]
        L.susp_batch_remove.argtypes = [vp, C.c_int32]
        L.susp_batch_step.argtypes = [vp, C.c_int64]
        L.susp_batch_stress.argtypes = [vp, C.c_int32, _PD, _PD]
        L.susp_batch_launch.argtypes = [vp, C.c_int32, C.c_int64]
        L.susp_batch_poll.argtypes = [vp, C.c_int32, _PI]
        L.susp_batch_launch_all.argtypes = [vp, C.c_int64]
        L.susp_batch_sim.argtypes = [vp, C.c_int32]
        L.susp_batch_sim.restype = vp
        L.susp_batch_bytes.argtypes = [vp]
        L.susp_batch_bytes.restype = C.c_size_t
        L.susp_batch_tune.argtypes = [vp, C.POINTER(Params), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.susp_batch_destroy.argtypes = [vp]
        _lib = L
    return _lib


def _chk(rc):
    if rc != 0:
        raise SuspError(rc, lib().susp_last_error().decode())
    return rc


def _pd(a):
    return None if a is None else a.ctypes.data_as(_PD)


def _pi(a):
    return None if a is None else a.ctypes.data_as(_PI)


def default_params() -> Params:
    p = Params()
    lib().susp_default_params(C.byref(p))
    return p


def make_params(box, radius=None, pos=None, vel=None, omega=None, precision=FP32, wall=None, **kw):
    """Build a Params with the paper's defaults; keyword names follow susp_params (wall: the
    per-sphere wall membership array for boundary = 1)."""
    p = default_params()
    p.lx, p.ly, p.lz = (int(v) for v in box)
    p.precision = int(precision)
    for k, v in kw.items():
        if not hasattr(p, k) or k == "wall":
            raise KeyError(k)
        setattr(p, k, v)
    keep = []
    if wall is not None:
        wall = np.ascontiguousarray(wall, dtype=np.int32)
        keep.append(wall)
        p.wall = _pi(wall)
    n = 0 if radius is None else len(radius)
    p.n = n
    if n:
        arrs = {}
        for name, a in (("pos", pos), ("vel", vel), ("omega", omega), ("radius", radius)):
            if a is None:
                continue
            a = np.ascontiguousarray(a, dtype=np.float64)
            arrs[name] = a
            keep.append(a)
            setattr(p, name, _pd(a))
    p._keep = keep  # keep the host arrays alive with the struct
    return p


def footprint_bytes(p: Params) -> int:
    nb = lib().susp_footprint_bytes(C.byref(p))
    if nb == 0:
        raise SuspError(EINVAL, lib().susp_last_error().decode())
    return int(nb)


class Simulation:
    """One simulation on the current HIP device and torch stream."""

    def __init__(self, p: Params, device="cuda", stream=None, own_workspace=True):
        import torch

        self.params = p
        self.nbytes = footprint_bytes(p)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.ws = None
        wptr = None
        if own_workspace:
            # PyTorch owns the device memory; the library carves its state out of it
            self.ws = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device)
            base = self.ws.data_ptr()
            wptr = (base + 255) // 256 * 256
        h = C.c_void_p()
        _chk(lib().susp_create(C.byref(p), C.c_void_p(self.stream.cuda_stream),
                               C.c_void_p(wptr) if wptr else None, self.nbytes, C.byref(h)))
        self.h = h
        self.n = p.n
        self.shape = (p.lz, p.ly, p.lx)

    def close(self):
        if getattr(self, "h", None):
            lib().susp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- stepping -----------------------------------------------------------------
    def step(self, n=1, check=True) -> int:
        rc = lib().susp_step(self.h, int(n))
        if check:
            _chk(rc)
        return rc

    def use_graphs(self, pairs=5):
        """Steps per replayed graph = 2 * pairs (0 or False: plain launches)."""
        _chk(lib().susp_use_graphs(self.h, int(pairs)))

    def profile(self, enable=True):
        _chk(lib().susp_profile(self.h, 1 if enable else 0))

    def profile_read(self):
        """(summed k_stream milliseconds, number of timed steps) since the last read."""
        ms = C.c_double(); n = C.c_int64()
        _chk(lib().susp_profile_read(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def profile_read_parts(self):
        """(summed k_links ms, summed k_stream ms, number of timed steps) since the last read."""
        ms = np.zeros(2); n = C.c_int64()
        _chk(lib().susp_profile_read_parts(self.h, _pd(ms), C.byref(n)))
        return float(ms[0]), float(ms[1]), n.value

    def stress(self):
        out = np.zeros((5, 6)); gg = np.zeros(2)
        _chk(lib().susp_stress(self.h, _pd(out), _pd(gg)))
        return out, gg

    def wall_force(self):
        """Mean force per step on the bottom and top walls since the last call (susp_wall_force)."""
        out = np.zeros(6)
        _chk(lib().susp_wall_force(self.h, _pd(out)))
        return out.reshape(2, 3)

    def contact_stats(self, nbins):
        """(hist[5][nbins] = rho, xi_N, xi_T, zeta_N, zeta_T; summary[12]) since the last
        call, then reset (susp_contact_stats)."""
        hist = np.zeros((5, nbins)); summ = np.zeros(12)
        _chk(lib().susp_contact_stats(self.h, int(nbins), _pd(hist), _pd(summ)))
        return hist, summ

    def contact_stats_noalloc(self, nbins):
        """contact_stats through the allocation-free entry point (static device staging,
        nbins <= 180; susp_contact_stats_noalloc)."""
        hist = np.zeros((5, nbins)); summ = np.zeros(12)
        _chk(lib().susp_contact_stats_noalloc(self.h, int(nbins), _pd(hist), _pd(summ)))
        return hist, summ

    # ---- state ----------------------------------------------------------------------
    def get_populations(self):
        f = np.zeros((19,) + self.shape)
        _chk(lib().susp_get_populations(self.h, _pd(f)))
        return f

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (19,) + self.shape
        _chk(lib().susp_set_populations(self.h, _pd(f)))

    def health(self):
        """(fluid node-steps above 0.3 c_s, largest |u| / c_s among them, relative drift of
        the conserved fluid mass + ledger) since the last call (susp_health)."""
        out = np.zeros(3)
        _chk(lib().susp_health(self.h, _pd(out)))
        return float(out[0]), float(out[1]), float(out[2])

    def get_accumulators(self):
        """Stress sums [5][6], their step count, the G', G'' sums and count, and the mass
        ledger (susp_get_accumulators)."""
        a = np.zeros(35)
        _chk(lib().susp_get_accumulators(self.h, _pd(a)))
        return a

    def set_accumulators(self, a):
        a = np.ascontiguousarray(a, np.float64).reshape(35)
        _chk(lib().susp_set_accumulators(self.h, _pd(a)))

    def get_state(self):
        """The whole state as bytes (susp_get_state): a checkpoint."""
        nb = C.c_size_t(0)
        _chk(lib().susp_get_state(self.h, None, C.byref(nb)))
        buf = np.zeros(nb.value, np.uint8)
        _chk(lib().susp_get_state(self.h, buf.ctypes.data_as(C.c_void_p), C.byref(nb)))
        return buf[:nb.value].tobytes()

    def set_state(self, state: bytes):
        buf = np.frombuffer(state, np.uint8).copy()
        _chk(lib().susp_set_state(self.h, buf.ctypes.data_as(C.c_void_p), len(buf)))

    def get_particles(self):
        n = self.n
        R = np.zeros((n, 3)); U = np.zeros((n, 3)); W = np.zeros((n, 3)); Q = np.zeros((n, 4))
        _chk(lib().susp_get_particles(self.h, _pd(R), _pd(U), _pd(W), _pd(Q)))
        return R, U, W, Q

    def set_particles(self, R=None, U=None, W=None, Q=None):
        conv = lambda a, w: None if a is None else np.ascontiguousarray(a, np.float64).reshape(-1, w)
        R, U, W, Q = conv(R, 3), conv(U, 3), conv(W, 3), conv(Q, 4)
        _chk(lib().susp_set_particles(self.h, _pd(R), _pd(U), _pd(W), _pd(Q)))

    def get_history(self):
        cnt = C.c_int32()
        _chk(lib().susp_get_history(self.h, 0, C.byref(cnt), None, None, None))
        k = cnt.value
        i = np.zeros(k, np.int32); j = np.zeros(k, np.int32); xi = np.zeros((k, 3))
        _chk(lib().susp_get_history(self.h, k, C.byref(cnt), _pi(i), _pi(j), _pd(xi)))
        return i, j, xi

    def set_history(self, i, j, xi):
        i = np.ascontiguousarray(i, np.int32); j = np.ascontiguousarray(j, np.int32)
        xi = np.ascontiguousarray(xi, np.float64).reshape(-1, 3)
        _chk(lib().susp_set_history(self.h, len(i), _pi(i), _pi(j), _pd(xi)))

    def clock(self):
        st = C.c_int64(); off = C.c_double()
        _chk(lib().susp_get_clock(self.h, C.byref(st), C.byref(off)))
        return st.value, off.value

    def set_clock(self, step):
        _chk(lib().susp_set_clock(self.h, int(step)))

    def hydro(self):
        n = self.n
        F = np.zeros((n, 3)); T = np.zeros((n, 3)); S = np.zeros((n, 6)); nl = np.zeros(n, np.int32)
        _chk(lib().susp_get_hydro(self.h, _pd(F), _pd(T), _pd(S), _pi(nl)))
        return F, T, S, nl

    def derived(self):
        out = np.zeros(10)
        _chk(lib().susp_get_derived(self.h, _pd(out)))
        keys = ("m0", "kn", "kt", "eta_n", "lub_delta", "F0", "debye_lambda", "eta0", "a_min", "a_max")
        return dict(zip(keys, out.tolist()))

    def lists(self, kind):
        nb = C.c_size_t(0)
        _chk(lib().susp_get_lists(self.h, int(kind), None, C.byref(nb)))
        buf = np.zeros(max(1, nb.value // 4), np.int32)
        nb2 = C.c_size_t(buf.nbytes)
        _chk(lib().susp_get_lists(self.h, int(kind), buf.ctypes.data_as(C.c_void_p), C.byref(nb2)))
        buf = buf[: nb.value // 4]
        p = self.params
        if kind == LIST_OWNER:
            return buf.reshape(self.shape)
        if kind == LIST_GHOST:
            return buf.reshape(2, p.lz, p.lx)
        if kind in (LIST_PAIRS, LIST_CONTACTS):
            return buf.reshape(-1, 2)
        if kind == LIST_LINKS:
            return buf.reshape(-1, 3)
        return buf


class _JobView(Simulation):
    """State getters of a job owned by a Batch (never destroys it)."""

    def __init__(self, handle, p: Params):
        self.h = C.c_void_p(handle)
        self.params = p
        self.n = p.n
        self.shape = (p.lz, p.ly, p.lx)
        self.stream = None
        self.ws = None

    def close(self):
        self.h = None


class Batch:
    """Many independent simulations on the current HIP device (one stream each).

    add() returns a slot, or None when the job's footprint does not fit in the remaining
    budget (admission refused; nothing changed)."""

    def __init__(self, max_jobs, hbm_budget, autotune=True):
        h = C.c_void_p()
        _chk(lib().susp_batch_create(int(max_jobs), int(hbm_budget), 1 if autotune else 0, C.byref(h)))
        self.h = h
        self.max_jobs = int(max_jobs)
        self._params = {}

    def add(self, p: Params):
        slot = C.c_int32(-1)
        rc = lib().susp_batch_add(self.h, C.byref(p), C.byref(slot))
        if rc == ENOMEM:
            return None
        _chk(rc)
        self._params[slot.value] = p
        return slot.value

    def remove(self, slot):
        _chk(lib().susp_batch_remove(self.h, int(slot)))
        self._params.pop(slot, None)

    def step(self, n, check=True):
        rc = lib().susp_batch_step(self.h, int(n))
        if check:
            _chk(rc)
        return rc

    def launch(self, slot, n):
        """Queue n steps of one job and return at once."""
        _chk(lib().susp_batch_launch(self.h, int(slot), int(n)))

    def launch_all(self, n):
        """Queue n steps of every job in lockstep (one launch per kernel over all jobs) and
        return at once; poll(slot) reports each job."""
        _chk(lib().susp_batch_launch_all(self.h, int(n)))

    def poll(self, slot):
        """(done, status): done once the job's queued steps have completed."""
        d = C.c_int32(0)
        rc = lib().susp_batch_poll(self.h, int(slot), C.byref(d))
        if rc not in (OK, EUNSTABLE):
            _chk(rc)
        return bool(d.value), rc

    def stress(self, slot):
        out = np.zeros((5, 6)); gg = np.zeros(2)
        _chk(lib().susp_batch_stress(self.h, int(slot), _pd(out), _pd(gg)))
        return out, gg

    def job(self, slot):
        h = lib().susp_batch_sim(self.h, int(slot))
        if not h:
            raise SuspError(EINVAL, "slot %d is free" % slot)
        return _JobView(h, self._params[slot])

    def bytes_in_use(self):
        return int(lib().susp_batch_bytes(self.h))

    def tune(self, p: Params):
        by = C.c_int32(); bz = C.c_int32()
        _chk(lib().susp_batch_tune(self.h, C.byref(p), C.byref(by), C.byref(bz)))
        return by.value, bz.value

    def close(self):
        if getattr(self, "h", None):
            lib().susp_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
