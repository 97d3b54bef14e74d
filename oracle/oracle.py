"""ctypes binding of the FP64 CPU oracle (``susp_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and by the
benchmark's CPU-baseline leg.  The GPU library never loads it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "susp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle (gcc, FP64, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "susp_oracle.h"))
    ):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-Wall",
             "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [
        ("lx", C.c_int32), ("ly", C.c_int32), ("lz", C.c_int32),
        ("tau", C.c_double), ("rho0", C.c_double),
        ("map_ratio", C.c_double), ("rho_p", C.c_double), ("kn", C.c_double),
        ("kt_ratio", C.c_double), ("mu", C.c_double), ("eta_n", C.c_double),
        ("lub_delta", C.c_double), ("lub_hc", C.c_double), ("lub_subtract_hc", C.c_int32),
        ("F0", C.c_double), ("debye_lambda", C.c_double), ("pair_cutoff", C.c_double),
        ("n_sub", C.c_int32), ("quasi2d", C.c_int32),
        ("shear_kind", C.c_int32), ("gamma_dot", C.c_double), ("g0_I", C.c_double),
        ("g0_F", C.c_double), ("period", C.c_int32), ("theta", C.c_double),
        ("ncyc_I", C.c_int32), ("ncyc_F", C.c_int32),
        ("wall_y", C.c_int32), ("wall_u_bot", C.c_double), ("wall_u_top", C.c_double),
        ("gx", C.c_double), ("gy", C.c_double), ("gz", C.c_double),
        ("contact_bins", C.c_int32), ("collision", C.c_int32), ("tau_bulk", C.c_double),
        ("tau_ghost", C.c_double), ("lub_implicit", C.c_int32), ("boundary", C.c_int32),
    ]


class Derived(C.Structure):
    _fields_ = [(k, C.c_double) for k in
                ("m0", "kn", "kt", "eta_n", "lub_delta", "F0", "debye_lambda", "eta0", "a_min", "a_max")]


_PD = C.POINTER(C.c_double)
_PI = C.POINTER(C.c_int32)


class Sim(C.Structure):
    _fields_ = [
        ("p", Params), ("d", Derived), ("nodes", C.c_int64),
        ("f", _PD), ("fn", _PD), ("own", _PI), ("np", C.c_int32),
        ("R", _PD), ("U", _PD), ("W", _PD), ("Q", _PD), ("a", _PD),
        ("m", _PD), ("I", _PD), ("amap", _PD),
        ("Fh", _PD), ("Th", _PD), ("Sh", _PD), ("nlinks", _PI), ("Frest", _PD), ("Trest", _PD),
        ("npairs", C.c_int32), ("pairs_cap", C.c_int32), ("pi", _PI), ("pj", _PI),
        ("nhist", C.c_int32), ("hist_cap", C.c_int32), ("hi", _PI), ("hj", _PI), ("hxi", _PD),
        ("gown", _PI),
        ("step", C.c_int64), ("s", C.c_double), ("ule", C.c_double), ("s_next", C.c_double),
        ("sig_last", (C.c_double * 6) * 5), ("sig_sum", (C.c_double * 6) * 5),
        ("sig_count", C.c_int64), ("gp_cos", C.c_double), ("gp_sin", C.c_double),
        ("gp_count", C.c_int64), ("ledger", C.c_double), ("flags", C.c_int32),
        ("nthreads", C.c_int32),
        ("cst", _PD), ("ctot", C.c_double * 6), ("csig", C.c_double * 6), ("csamples", C.c_int64),
        ("wall", _PI), ("wforce", (C.c_double * 3) * 2), ("wcount", C.c_int64), ("wspeed", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        L.orc_create.restype = C.POINTER(Sim)
        L.orc_create.argtypes = [C.POINTER(Params), C.c_int32, _PD, _PD, _PD, _PD]
        L.orc_destroy.argtypes = [C.POINTER(Sim)]
        L.orc_step.argtypes = [C.POINTER(Sim), C.c_int64]
        L.orc_step.restype = C.c_int
        L.orc_remap.argtypes = [C.POINTER(Sim)]
        L.orc_set_history.argtypes = [C.POINTER(Sim), C.c_int32, _PI, _PI, _PD]
        L.orc_stress.argtypes = [C.POINTER(Sim), _PD, _PD]
        L.orc_protocol.argtypes = [C.POINTER(Params), C.c_int64, _PD, _PD]
        L.orc_feq.argtypes = [C.c_double] * 4 + [_PD]
        L.orc_minimage.argtypes = [C.POINTER(Params), C.c_double, C.c_double, C.c_double,
                                   C.c_double, _PD, _PI]
        L.orc_resolve.argtypes = [C.POINTER(Params), C.c_int32, _PD, C.POINTER(Derived)]
        L.orc_lubrication.argtypes = [C.POINTER(Params), C.POINTER(Derived), C.c_double,
                                      C.c_double] + [_PD] * 10
        L.orc_contact.argtypes = [C.POINTER(Params), C.POINTER(Derived), C.c_double,
                                  C.c_double] + [_PD] * 5 + [C.c_double] + [_PD] * 5
        L.orc_contact.restype = C.c_int
        L.orc_dlvo.argtypes = [C.POINTER(Params), C.POINTER(Derived), C.c_double, C.c_double,
                               _PD, _PD]
        L.orc_lattice.argtypes = [_PI, _PI, _PI, _PD, _PI]
        L.orc_contact_stats.argtypes = [C.POINTER(Sim), C.c_int32, _PD, _PD]
        L.orc_contact_stats.restype = C.c_int
        L.orc_sym3_eigen.argtypes = [_PD, _PD]
        L.orc_set_walls.argtypes = [C.POINTER(Sim), _PI]
        L.orc_set_walls.restype = C.c_int
        L.orc_wall_speed.argtypes = [C.POINTER(Params), C.c_int64]
        L.orc_wall_speed.restype = C.c_double
        L.orc_wall_force.argtypes = [C.POINTER(Sim), _PD]
        L.orc_lub_squeeze.argtypes = [C.POINTER(Params), C.POINTER(Derived), C.c_double, C.c_double, _PD]
        L.orc_lub_squeeze.restype = C.c_double
        L.orc_implicit_solve.argtypes = [C.c_int32, _PD, _PI, _PD, C.c_int32, _PI, _PI, _PD, _PD, _PD,
                                         C.c_double, C.c_int32, _PD]
        L.orc_gg_weight.argtypes = [C.POINTER(Params), C.c_int64, _PD, _PD]
        L.orc_gg_weight.restype = C.c_int
        L.orc_gg_moduli.argtypes = [C.POINTER(Params), C.c_double, C.c_double, C.c_int64, _PD]
        L.orc_gg_series.argtypes = [C.POINTER(Params), C.c_int64, C.c_int64, _PD, _PD]
        L.orc_quat_step.argtypes = [_PD, _PD, C.c_double]
        _lib = L
    return _lib


def _pd(a):
    return a.ctypes.data_as(_PD)


def _pi(a):
    return a.ctypes.data_as(_PI)


DEFAULTS = dict(
    tau=1.0, rho0=1.0, map_ratio=0.95, rho_p=1.0, kn=-1.0, kt_ratio=0.5, mu=1.0, eta_n=-1.0,
    lub_delta=-1.0, lub_hc=0.5, lub_subtract_hc=1, F0=-1.0, debye_lambda=-1.0, pair_cutoff=1.0,
    n_sub=8, quasi2d=0, shear_kind=0, gamma_dot=0.0, g0_I=0.0, g0_F=0.0, period=1, theta=0.0,
    ncyc_I=0, ncyc_F=0, wall_y=0, wall_u_bot=0.0, wall_u_top=0.0, gx=0.0, gy=0.0, gz=0.0,
    contact_bins=0, collision=0, tau_bulk=1.0, tau_ghost=1.0, lub_implicit=0, boundary=0,
)


def make_params(**kw) -> Params:
    d = dict(DEFAULTS)
    unknown = set(kw) - set(d) - {"lx", "ly", "lz"}
    if unknown:
        raise KeyError("unknown oracle parameters: %s" % sorted(unknown))
    d.update(kw)
    p = Params()
    for k, v in d.items():
        setattr(p, k, v)
    return p


def lattice():
    cx = np.zeros(19, np.int32); cy = np.zeros(19, np.int32); cz = np.zeros(19, np.int32)
    w = np.zeros(19); opp = np.zeros(19, np.int32)
    lib().orc_lattice(_pi(cx), _pi(cy), _pi(cz), _pd(w), _pi(opp))
    return np.stack([cx, cy, cz], 1), w, opp


def feq(rho, u):
    out = np.zeros(19)
    lib().orc_feq(float(rho), float(u[0]), float(u[1]), float(u[2]), _pd(out))
    return out


def protocol(params: Params, t: int):
    s = C.c_double(); u = C.c_double()
    lib().orc_protocol(C.byref(params), int(t), C.byref(s), C.byref(u))
    return s.value, u.value


def minimage(params: Params, s, d):
    out = np.zeros(3); k = np.zeros(1, np.int32)
    lib().orc_minimage(C.byref(params), float(s), float(d[0]), float(d[1]), float(d[2]),
                       _pd(out), _pi(k))
    return out, int(k[0])


def resolve(params: Params, radius) -> Derived:
    r = np.ascontiguousarray(radius, dtype=np.float64)
    d = Derived()
    lib().orc_resolve(C.byref(params), len(r), _pd(r), C.byref(d))
    return d


def _v3(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(3))


def lubrication(params, derived, ai, aj, d, Ui, Uj, Wi, Wj):
    Fi = np.zeros(3); Ti = np.zeros(3); Tj = np.zeros(3); Si = np.zeros(6); Sj = np.zeros(6)
    args = [_v3(v) for v in (d, Ui, Uj, Wi, Wj)]
    lib().orc_lubrication(C.byref(params), C.byref(derived), float(ai), float(aj),
                          *[_pd(a) for a in args], _pd(Fi), _pd(Ti), _pd(Tj), _pd(Si), _pd(Sj))
    return Fi, Ti, Tj, Si, Sj


def contact(params, derived, ai, aj, d, Ui, Uj, Wi, Wj, dt, xi):
    xi = _v3(xi).copy()
    Fi = np.zeros(3); Ti = np.zeros(3); Tj = np.zeros(3); Fn = np.zeros(3)
    args = [_v3(v) for v in (d, Ui, Uj, Wi, Wj)]
    on = lib().orc_contact(C.byref(params), C.byref(derived), float(ai), float(aj),
                           *[_pd(a) for a in args], float(dt), _pd(xi), _pd(Fi), _pd(Ti),
                           _pd(Tj), _pd(Fn))
    return on, xi, Fi, Ti, Tj, Fn


def dlvo(params, derived, ai, aj, d):
    Fi = np.zeros(3)
    lib().orc_dlvo(C.byref(params), C.byref(derived), float(ai), float(aj), _pd(_v3(d)), _pd(Fi))
    return Fi


def lub_squeeze(params, derived, ai, aj, d):
    return lib().orc_lub_squeeze(C.byref(params), C.byref(derived), float(ai), float(aj), _pd(_v3(d)))


def implicit_solve(m, fixed, b, pi, pj, zeta, nvec, shift, dt, sweeps, U0):
    """The substep's velocities with implicit squeeze terms (orc_implicit_solve)."""
    m = np.ascontiguousarray(m, np.float64); n = len(m)
    fixed = np.ascontiguousarray(fixed, np.int32)
    b = np.ascontiguousarray(b, np.float64).reshape(n, 3)
    pi = np.ascontiguousarray(pi, np.int32); pj = np.ascontiguousarray(pj, np.int32)
    zeta = np.ascontiguousarray(zeta, np.float64)
    nvec = np.ascontiguousarray(nvec, np.float64).reshape(-1, 3)
    shift = np.ascontiguousarray(shift, np.float64).reshape(-1, 3)
    U = np.ascontiguousarray(U0, np.float64).reshape(n, 3).copy()
    lib().orc_implicit_solve(n, _pd(m), _pi(fixed), _pd(b), len(pi), _pi(pi), _pi(pj), _pd(zeta),
                             _pd(nvec), _pd(shift), float(dt), int(sweeps), _pd(U))
    return U


def gg_series(params: Params, t0: int, sxy):
    """{G', G''} of eqs. (17)-(18) from the shear-stress history sxy (sxy[k]: step t0 + k)."""
    a = np.ascontiguousarray(sxy, np.float64).reshape(-1)
    gg = np.zeros(2)
    lib().orc_gg_series(C.byref(params), int(t0), len(a), _pd(a), _pd(gg))
    return gg


def quat_step(q, W, dt):
    """One substep's orientation update of a sphere with angular velocity W."""
    q = np.ascontiguousarray(q, np.float64).reshape(4).copy()
    lib().orc_quat_step(_pd(q), _pd(_v3(W)), float(dt))
    return q


def wall_speed(params: Params, t: int) -> float:
    return lib().orc_wall_speed(C.byref(params), int(t))


def sym3_eigen(a6):
    """Eigenvalues (descending) of the symmetric 3x3 matrix xx yy zz xy xz yz."""
    a = np.ascontiguousarray(a6, np.float64).reshape(6)
    ev = np.zeros(3)
    lib().orc_sym3_eigen(_pd(a), _pd(ev))
    return ev


class Oracle:
    """One simulation held by the C oracle; arrays are live numpy views of its memory."""

    def __init__(self, params: Params, pos=None, vel=None, omega=None, radius=None, wall=None):
        self.params = params
        pos = np.zeros((0, 3)) if pos is None else np.ascontiguousarray(pos, np.float64).reshape(-1, 3)
        n = pos.shape[0]
        vel = np.zeros((n, 3)) if vel is None else np.ascontiguousarray(vel, np.float64).reshape(-1, 3)
        omega = np.zeros((n, 3)) if omega is None else np.ascontiguousarray(omega, np.float64).reshape(-1, 3)
        radius = np.zeros(0) if radius is None else np.ascontiguousarray(radius, np.float64).reshape(-1)
        self._keep = (pos, vel, omega, radius)
        self.ptr = lib().orc_create(C.byref(params), n, _pd(pos), _pd(vel), _pd(omega), _pd(radius))
        self.s = self.ptr.contents
        # the lattice loop is split over z-planes: no more threads than planes, and one thread
        # per 4096 nodes at most (a tiny box otherwise spends its steps in thread barriers)
        nodes = int(params.lx) * int(params.ly) * int(params.lz)
        self.s.nthreads = max(1, min(int(self.s.nthreads), int(params.lz), nodes // 4096))
        if wall is not None:
            wall = np.ascontiguousarray(wall, np.int32).reshape(-1)
            if lib().orc_set_walls(self.ptr, _pi(wall)):
                raise ValueError("wall spheres must keep pair_cutoff / 2 from their box face")

    def __del__(self):
        try:
            if getattr(self, "ptr", None):
                lib().orc_destroy(self.ptr)
                self.ptr = None
        except Exception:
            pass

    # ---- views -------------------------------------------------------------------
    def _arr(self, ptr, shape, dtype=np.float64):
        n = int(np.prod(shape))
        if n == 0:
            return np.zeros(shape, dtype)
        return np.ctypeslib.as_array(ptr, shape=(n,)).reshape(shape)

    @property
    def f(self):
        p = self.params
        return self._arr(self.s.f, (19, p.lz, p.ly, p.lx))

    @property
    def own(self):
        p = self.params
        return self._arr(self.s.own, (p.lz, p.ly, p.lx), np.int32)

    @property
    def np(self):
        return self.s.np

    def part(self, name):
        width = {"R": 3, "U": 3, "W": 3, "Q": 4, "a": None, "m": None, "I": None, "amap": None,
                 "Fh": 3, "Th": 3, "Sh": 9, "Frest": 3, "Trest": 3}[name]
        shape = (self.s.np,) if width is None else (self.s.np, width)
        return self._arr(getattr(self.s, name), shape)

    @property
    def nlinks(self):
        return self._arr(self.s.nlinks, (self.s.np,), np.int32)

    def pairs(self):
        n = self.s.npairs
        return (self._arr(self.s.pi, (n,), np.int32).copy(), self._arr(self.s.pj, (n,), np.int32).copy())

    def history(self):
        n = self.s.nhist
        return (self._arr(self.s.hi, (n,), np.int32).copy(), self._arr(self.s.hj, (n,), np.int32).copy(),
                self._arr(self.s.hxi, (n, 3)).copy())

    def set_history(self, i, j, xi):
        i = np.ascontiguousarray(i, np.int32); j = np.ascontiguousarray(j, np.int32)
        xi = np.ascontiguousarray(xi, np.float64).reshape(-1, 3)
        lib().orc_set_history(self.ptr, len(i), _pi(i), _pi(j), _pd(xi))

    @property
    def gown(self):
        p = self.params
        return self._arr(self.s.gown, (2, p.lz, p.lx), np.int32)

    def remap(self):
        lib().orc_remap(self.ptr)

    # ---- stepping and observables ----------------------------------------------------
    def step(self, n=1) -> int:
        return lib().orc_step(self.ptr, int(n))

    def stress(self):
        out = np.zeros((5, 6)); gg = np.zeros(2)
        lib().orc_stress(self.ptr, _pd(out), _pd(gg))
        return out, gg

    def wall_force(self):
        """Mean force per step on the bottom and top walls since the last call, then reset."""
        out = np.zeros(6)
        lib().orc_wall_force(self.ptr, _pd(out))
        return out.reshape(2, 3)

    def contact_stats(self, nbins):
        """(hist[5][nbins] = rho, xi_N, xi_T, zeta_N, zeta_T; summary[12]) since the last
        call, then reset (see orc_contact_stats)."""
        hist = np.zeros((5, nbins)); summ = np.zeros(12)
        rc = lib().orc_contact_stats(self.ptr, int(nbins), _pd(hist), _pd(summ))
        if rc:
            raise ValueError("nbins must equal the simulation's contact_bins")
        return hist, summ

    def sig_last(self):
        return np.array([[self.s.sig_last[k][c] for c in range(6)] for k in range(5)])

    def moments(self):
        """Density and velocity of every node from the stored populations."""
        cvec, _, _ = lattice()
        f = self.f
        rho = f.sum(0)
        j = np.tensordot(cvec.T.astype(np.float64), f, axes=([1], [0]))
        return rho, j / rho
