"""Shared helpers of the GPU parity tests (not collected by pytest).

States are produced by the oracle and rounded on the host exactly as the library rounds
them when they are loaded, so that the oracle and the GPU start from identical values.
"""
import math

import numpy as np

from oracle import oracle as O
from paper_1904_02929_amd import synth

ORACLE_KEYS = set(O.DEFAULTS) - {"wall_y", "wall_u_bot", "wall_u_top", "gx", "gy", "gz"}


def weights():
    _, w, _ = O.lattice()
    return w


def rounded(f, precision, rho0=1.0, k=10):
    """Populations as the library stores them: deviations in FP64, FP32, or FP16 of
    (n - w rho0) / w * 2^k."""
    w = weights()[:, None, None, None] * rho0
    if precision == 0:
        return np.array(f, dtype=np.float64)
    d = (f - w).astype(np.float32)
    if precision == 1:
        return w + d.astype(np.float64)
    wq = weights()
    sc = np.array([np.float32(2.0 ** k / x) for x in wq], np.float32)[:, None, None, None]
    isc = np.array([np.float32(x * 2.0 ** -k) for x in wq], np.float32)[:, None, None, None]
    h = (d * sc).astype(np.float16)
    return w + (h.astype(np.float32) * isc).astype(np.float64)


def oracle_for(box, kw, pos, vel, omega, radius):
    p = O.make_params(lx=box[0], ly=box[1], lz=box[2], **{k: v for k, v in kw.items() if k in ORACLE_KEYS})
    return O.Oracle(p, pos, vel, omega, radius)


def gpu_for(box, kw, pos, vel, omega, radius, precision):
    from paper_1904_02929_amd import susp
    gk = {k: v for k, v in kw.items() if k in ORACLE_KEYS or k in ("fp16_exp", "brick_y", "brick_z")}
    p = susp.make_params(box, radius=radius, pos=pos, vel=vel, omega=omega, precision=precision, **gk)
    return susp.Simulation(p)


def load_oracle_state(o, g, precision):
    """Round the oracle's state to the storage precision and load it into both sides."""
    f = rounded(o.f, precision, o.params.rho0)
    o.f[...] = f
    R, U, W, Q = o.part("R").copy(), o.part("U").copy(), o.part("W").copy(), o.part("Q").copy()
    g.set_clock(int(o.s.step))
    g.set_particles(R, U, W, Q)
    g.set_populations(f)
    hi, hj, hx = o.history()
    g.set_history(hi, hj, hx)
    g.set_accumulators(oracle_accumulators(o))


def oracle_accumulators(o):
    """The oracle's running sums in the library's accumulator layout: stress sums [5][6],
    their count, the G', G'' sums and count, the mass ledger."""
    s = o.s
    acc = [s.sig_sum[k][c] for k in range(5) for c in range(6)]
    acc += [float(s.sig_count), s.gp_cos, s.gp_sin, float(s.gp_count), s.ledger]
    return np.array(acc)


def moments(f):
    c, _, _ = O.lattice()
    rho = f.sum(0)
    j = np.tensordot(c.T.astype(np.float64), f, axes=([1], [0]))
    return rho, j / rho


def equilibrium(rho, u):
    """Second-order D3Q19 equilibrium of every node, [19][nodes] (written out here from
    the lattice's velocities and weights, independent of both implementations)."""
    c, w, _ = O.lattice()
    c = c.astype(np.float64)
    cu = c @ u  # [19][nodes]
    uu = (u * u).sum(0)
    return w[:, None] * rho[None, :] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu[None, :])


def rel(a, b, floor=0.0):
    """max|a - b| / max(max|b|, floor): relative error with an absolute floor for
    quantities whose reference is (close to) zero."""
    a = np.asarray(a, float); b = np.asarray(b, float)
    if not a.size:
        return 0.0
    scale = max(float(np.abs(b).max()), floor)
    if scale == 0.0:
        return float(np.abs(a - b).max())
    return float(np.abs(a - b).max() / scale)


def contacts_at_start(o_params, R, radius, s, pairs):
    out = []
    for i, j in pairs:
        d, _ = O.minimage(o_params, s, R[i] - R[j])
        r = math.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
        if r - radius[i] - radius[j] < 0.0:
            out.append((int(i), int(j)))
    return out


def cell_list(box, R, radius, cutoff=1.0):
    """Cell list by its definition: cell = floor(R * n/L) per axis (n cells of width at
    least 2 a_max + cutoff), ids ascending inside each cell."""
    rc = 2.0 * max(radius) + cutoff + 1e-6
    nc = [min(64, max(1, int(math.floor(L / rc)))) for L in box]
    inv = [nc[c] / float(box[c]) for c in range(3)]
    cells = []
    for i in range(len(R)):
        a = [min(nc[c] - 1, max(0, int(math.floor(R[i][c] * inv[c])))) for c in range(3)]
        cells.append(a[0] + nc[0] * (a[1] + nc[1] * a[2]))
    cells = np.array(cells)
    order = np.lexsort((np.arange(len(R)), cells))
    start = np.searchsorted(cells[order], np.arange(nc[0] * nc[1] * nc[2] + 1))
    return start.astype(np.int32), order.astype(np.int32)


def dense_workload(box=(41, 48, 37), phi=0.45, seed=7, gd=1e-3):
    rng = np.random.default_rng(seed)
    n = synth.count_for_phi3(phi, box, 4.5, 6.3)
    rad = synth.bidisperse_radii(n, 4.5, 6.3, rng)
    pos = synth.pack(box, rad, rng, margin=0.05)
    vel, om = synth.affine_start(pos, rad, gd, box[1])
    return box, pos, vel, om, rad, dict(shear_kind=1, gamma_dot=gd)
