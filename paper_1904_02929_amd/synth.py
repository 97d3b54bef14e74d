"""Seeded synthetic inputs for the sheared-suspension step.

This module only draws inputs: sphere radii, non-overlapping positions, initial velocities
and the workload descriptions.  It performs none of the method's arithmetic (no lattice
Boltzmann, no contact or lubrication forces), so both the GPU library and the CPU oracle can
be fed from it without sharing any of the method.

Workloads follow the paper's parameters: bidisperse 1:1 mixtures with a_max = 1.4 a_min
(Sec. 2, bidispersity), the 3D volume fraction phi3 = 2 N pi (a_max^3 + a_min^3) / (3V) and
the monolayer area fraction phi = N pi (a_max^2 + a_min^2) / (2 Lx Ly) (Secs. 3.1 and 4.1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

try:  # neighbour search for the packing relaxation
    from scipy.spatial import cKDTree
except Exception:  # pragma: no cover - scipy is present in the supported image
    cKDTree = None


def count_for_phi3(phi: float, box, a_small: float, a_large: float) -> int:
    """Number of spheres (1:1 bidisperse) giving volume fraction phi in the box."""
    V = float(box[0]) * box[1] * box[2]
    return int(round(phi * 3.0 * V / (2.0 * math.pi * (a_small**3 + a_large**3))))


def count_for_area(phi: float, box, a: float) -> int:
    """Number of equal spheres of radius a giving monolayer area fraction phi."""
    return int(round(phi * box[0] * box[1] / (math.pi * a * a)))


def bidisperse_radii(n: int, a_small: float, a_large: float, rng: np.random.Generator):
    r = np.where(np.arange(n) < n // 2, a_small, a_large).astype(np.float64)
    rng.shuffle(r)
    return r


def _pairs(pos, box, cutoff, planar):
    pts = pos[:, :2] if planar else pos
    tree = cKDTree(pts % (box[:2] if planar else box), boxsize=box[:2] if planar else box)
    return tree.query_pairs(cutoff, output_type="ndarray")


def _overlap_forces(pos, rad, box, pr, planar):
    i, j = pr[:, 0], pr[:, 1]
    d = pos[i] - pos[j]
    d -= box * np.round(d / box)
    if planar:
        d[:, 2] = 0.0
    r = np.sqrt((d * d).sum(1))
    ov = rad[i] + rad[j] - r
    m = ov > 0
    F = np.zeros_like(pos)
    worst = 0.0
    if m.any():
        i, j, d, r, ov = i[m], j[m], d[m], r[m], ov[m]
        r = np.where(r > 1e-12, r, 1e-12)
        fij = ov[:, None] * d / r[:, None]
        np.add.at(F, i, fij)
        np.add.at(F, j, -fij)
        worst = float(ov.max())
    return F, worst


def pack(box, radii, rng: np.random.Generator, margin: float = 0.1, z_fixed=None,
         tol: float = 1e-10, max_iter: int = 200000):
    """Random non-overlapping positions in a periodic box.

    Spheres are dropped uniformly at random and the harmonic overlap energy
    sum 1/2 max(0, r_i + r_j - |d_ij|)^2 of the radii inflated by ``margin``/2 is minimised
    with FIRE (Bitzek et al. 2006) until the largest overlap is below ``tol``.  With
    ``z_fixed`` all centres stay in the plane z = z_fixed (monolayer).
    """
    if cKDTree is None:
        raise RuntimeError("scipy is required for the packing generator")
    box = np.asarray(box, dtype=np.float64)
    n = len(radii)
    if n == 0:
        return np.zeros((0, 3))
    planar = z_fixed is not None
    rad = np.asarray(radii, dtype=np.float64) + 0.5 * margin
    pos = rng.random((n, 3)) * box
    if planar:
        pos[:, 2] = z_fixed
    skin = 0.5
    cut = 2.0 * rad.max() + skin
    pr = _pairs(pos, box, cut, planar)
    ref = pos.copy()
    v = np.zeros_like(pos)
    dt, dtmax, alpha, npos = 0.05, 0.5, 0.1, 0
    for it in range(max_iter):
        moved = pos - ref
        moved -= box * np.round(moved / box)
        if np.abs(moved).max() > 0.5 * skin:
            pr = _pairs(pos, box, cut, planar)
            ref = pos.copy()
        F, worst = _overlap_forces(pos, rad, box, pr, planar)
        if worst <= tol:
            return pos % box
        P = float((F * v).sum())
        if P > 0:
            fn = np.sqrt((F * F).sum()) + 1e-300
            vn = np.sqrt((v * v).sum())
            v = (1.0 - alpha) * v + alpha * vn * F / fn
            npos += 1
            if npos > 5:
                dt = min(dt * 1.1, dtmax)
                alpha *= 0.99
        else:
            v[:] = 0.0
            dt *= 0.5
            alpha = 0.1
            npos = 0
        v += dt * F
        if planar:
            v[:, 2] = 0.0
        pos += dt * v
    raise RuntimeError("packing did not converge")


@dataclass
class Workload:
    """A synthetic suspension: box, spheres, protocol and the solver parameters."""
    name: str
    box: tuple
    pos: np.ndarray
    vel: np.ndarray
    omega: np.ndarray
    radius: np.ndarray
    params: dict = field(default_factory=dict)
    wall: np.ndarray = None  # per-sphere wall membership (0 free, 1 bottom, 2 top) with walls

    @property
    def n(self):
        return len(self.radius)


def affine_start(pos, radius, gamma_dot: float, ly: int):
    """Velocities that follow the imposed shear u_x = gdot (y - (ly-1)/2); spin -gdot/2."""
    n = len(radius)
    vel = np.zeros((n, 3))
    om = np.zeros((n, 3))
    if n:
        vel[:, 0] = gamma_dot * (pos[:, 1] - 0.5 * (ly - 1))
        om[:, 2] = -0.5 * gamma_dot
    return vel, om


def single_sphere(L: int = 32, a: float = 4.5, gamma_dot: float = 1e-4) -> Workload:
    """One sphere at the box centre in simple shear (32^3, a = 4.5)."""
    c = 0.5 * (L - 1)
    pos = np.array([[c, c, c]])
    rad = np.array([a])
    return Workload("single_sphere_%d" % L, (L, L, L), pos, np.zeros((1, 3)), np.zeros((1, 3)), rad,
                    dict(shear_kind=1, gamma_dot=gamma_dot))


def bulk3d(L: int, phi: float, gamma_dot: float, seed: int, a_small=4.5, a_large=6.3,
           margin: float = 0.1) -> Workload:
    """Bidisperse 3D suspension in an L^3 box under simple Lees-Edwards shear."""
    rng = np.random.default_rng(seed)
    box = (L, L, L)
    n = count_for_phi3(phi, box, a_small, a_large)
    rad = bidisperse_radii(n, a_small, a_large, rng)
    pos = pack(box, rad, rng, margin=margin)
    vel, om = affine_start(pos, rad, gamma_dot, L)
    return Workload("bulk3d_%d_phi%.2f" % (L, phi), box, pos, vel, om, rad,
                    dict(shear_kind=1, gamma_dot=gamma_dot))


def monolayer(L: int, lz: int, phi: float, seed: int, a: float = 4.5, g0_I=0.1, g0_F=1e-3,
              theta=0.0, period=2000, ncyc_I=3, ncyc_F=2, margin: float = 0.1) -> Workload:
    """Quasi-2D monolayer of equal spheres at mid-height under oscillatory shear."""
    rng = np.random.default_rng(seed)
    box = (L, L, lz)
    n = count_for_area(phi, box, a)
    rad = np.full(n, a)
    pos = pack(box, rad, rng, margin=margin, z_fixed=0.5 * lz)
    om_rate = 2.0 * math.pi / period * g0_I * math.sin(theta)
    vel, om = affine_start(pos, rad, om_rate, L)
    return Workload("monolayer_%d_phi%.2f" % (L, phi), box, pos, vel, om, rad,
                    dict(shear_kind=2, g0_I=g0_I, g0_F=g0_F, theta=theta, period=period,
                         ncyc_I=ncyc_I, ncyc_F=ncyc_F, quasi2d=1))


def walled3d(L: int, phi: float, gamma_dot: float, seed: int, a_small=4.5, a_large=6.3,
             a_wall=4.5, margin: float = 0.1) -> Workload:
    """Bidisperse 3D suspension sheared by two moving walls of spheres (boundary 1).

    Each wall is a square layer of spheres of radius a_wall, centres 0.6 lattice units plus
    a_wall from the box face (the pair cutoff is 1), spaced 2 a_wall + 1.2 apart in x and z
    (rounded to divide L), the top layer shifted by half a spacing in x.  The free spheres
    fill the gap between the two layers at volume fraction phi of the gap's volume; packed in
    a box periodic in y, those within margin of the gap's faces are dropped.
    """
    rng = np.random.default_rng(seed)
    box = (L, L, L)
    yb, yt = a_wall + 0.6, L - a_wall - 0.6
    nw = max(1, int(L // (2 * a_wall + 1.2)))
    sp = L / nw
    wall_pos = []
    for y, shift, m in ((yb, 0.0, 1), (yt, 0.5 * sp, 2)):
        for i in range(nw):
            for k in range(nw):
                wall_pos.append((((i + 0.5) * sp + shift) % L, y, (k + 0.5) * sp, m))
    wall_pos = np.array(wall_pos)
    lo, hi = yb + a_wall + margin, yt - a_wall - margin
    gap = (L, hi - lo, L)
    n = count_for_phi3(phi, gap, a_small, a_large)
    rad = bidisperse_radii(n, a_small, a_large, rng)
    pos = pack(gap, rad, rng, margin=margin)
    keep = (pos[:, 1] - rad > margin) & (pos[:, 1] + rad < gap[1] - margin)
    pos, rad = pos[keep], rad[keep]
    pos[:, 1] += lo
    allpos = np.concatenate([wall_pos[:, :3], pos])
    allrad = np.concatenate([np.full(len(wall_pos), a_wall), rad])
    wall = np.concatenate([wall_pos[:, 3].astype(np.int32), np.zeros(len(rad), np.int32)])
    vel, om = affine_start(allpos, allrad, gamma_dot, L)
    vel[wall > 0] = 0.0
    om[wall > 0] = 0.0
    return Workload("walled3d_%d_phi%.2f" % (L, phi), box, allpos, vel, om, allrad,
                    dict(shear_kind=1, gamma_dot=gamma_dot, boundary=1), wall=wall)
