// fluid.hip -- lattice-Boltzmann kernels for gfx950.
//
//  k_lbm      fused pull-stream + moving bounce-back + BGK collision + link forces + fluid
//             stress partials (App. A eqs. 3-10), one thread per node, x fastest.
//  k_ghosts   Lees-Edwards ghost planes y=-1 and y=ly: geometric owner test of each ghost
//             point, else linear interpolation of the Galilean-corrected post-collision
//             row shifted by the offset (Wagner & Pagonabarraga).
//  helpers    equilibrium fill, FP64 <-> storage conversion, link enumeration.
#include "susp_impl.h"

namespace susp {

// ---------------------------------------------------------------------------------------
// FP64 surface velocity of sphere p at lever l = r_b - R_img (eq. 8), image index k.
__device__ inline void surf_vel(const double *U, const double *W, int p, int k, double ule,
                                double lx, double ly, double lz, double &ux, double &uy,
                                double &uz) {
  const double w0 = W[3 * p], w1 = W[3 * p + 1], w2 = W[3 * p + 2];
  ux = U[3 * p] + k * ule + (w1 * lz - w2 * ly);
  uy = U[3 * p + 1] + (w2 * lx - w0 * lz);
  uz = U[3 * p + 2] + (w0 * ly - w1 * lx);
}

template <class T> __device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------------------
struct LbmArgs {
  const void *fin;
  void *fout;
  size_t plane;
  const int32_t *own;
  const int32_t *gown;
  const void *gval;
  const double *R, *U, *W;
  double *hyd;
  double *pineq;
  int64_t nodes;
  int lx, ly, lz;
  int nblk, per_xcd;
  Box b;
  double rho0, omega;
  float tab[2 * NQ];
};

// Per-lane accumulation of the links of one sphere; flushed when the sphere changes.
struct LinkAcc {
  int p;
  double v[HYD];
};

__device__ inline void link_flush_atomic(double *hyd, const LinkAcc &a) {
  for (int c = 0; c < HYD; ++c) unsafeAtomicAdd(&hyd[(size_t)a.p * HYD + c], a.v[c]);
}

template <class ST>
__global__ __launch_bounds__(LBM_BLOCK) void k_lbm(LbmArgs A) {
  using CT = typename Store<ST>::CT;
  const ST *fin = (const ST *)A.fin;
  ST *fout = (ST *)A.fout;
  const CT *gval = (const CT *)A.gval;
  // XCD-aware tile order: consecutive hardware blocks are dealt round-robin to the 8 XCDs;
  // give each XCD a contiguous range of tiles so neighbouring rows share its L2.
  const int hb = blockIdx.x;
  const int xcd = hb & 7, slot = hb >> 3;
  int blk = xcd * A.per_xcd + slot;
  const bool blk_ok = blk < A.nblk;
  if (!blk_ok) blk = 0;
  const int64_t node = (int64_t)blk * LBM_BLOCK + threadIdx.x;
  const bool valid = blk_ok && node < A.nodes;
  const int lx = A.lx, ly = A.ly, lz = A.lz;
  int x = 0, y = 0, z = 0;
  int own = -2;
  if (valid) {
    own = A.own[node];
    x = (int)(node % lx);
    int64_t yz = node / lx;
    y = (int)(yz % ly);
    z = (int)(yz / ly);
  }
  const bool fluid = own == -1;
  LinkAcc acc;
  acc.p = -1;
#pragma unroll
  for (int c = 0; c < HYD; ++c) acc.v[c] = 0.0;
  CT pn[6] = {0, 0, 0, 0, 0, 0};
  if (fluid) {
    CT n[NQ];
    n[0] = Store<ST>::ld(fin, node, 0, A.tab);
#pragma unroll
    for (int q = 1; q < NQ; ++q) {
      int px = x - cx(q), py = y - cy(q), pz = z - cz(q);
      px = px < 0 ? px + lx : (px >= lx ? px - lx : px);
      pz = pz < 0 ? pz + lz : (pz >= lz ? pz - lz : pz);
      int so;
      CT val = 0;
      if (cy(q) != 0 && (py < 0 || py >= ly)) {
        const int g = py < 0 ? 0 : 1;
        const int gi = (g * lz + pz) * lx + px;
        so = A.gown[gi];
        if (so < 0) val = gval[(size_t)((g * 5 + gslot(q)) * lz + pz) * lx + px];
      } else {
        const int64_t src = px + (int64_t)lx * (py + (int64_t)ly * pz);
        so = A.own[src];
        if (so < 0) val = Store<ST>::ld(fin, (size_t)q * A.plane + src, q, A.tab);
      }
      if (so < 0) {
        n[q] = val;
      } else {
        // eqs. (7)-(8): bounce-back off the surface halfway along the link, FP64
        const int p = so;
        double dx, dy, dz;
        int k;
        minimage(A.b, (double)(x - cx(q)) - A.R[3 * p], (double)(y - cy(q)) - A.R[3 * p + 1],
                 (double)(z - cz(q)) - A.R[3 * p + 2], dx, dy, dz, k);
        const double lvx = dx + 0.5 * cx(q), lvy = dy + 0.5 * cy(q), lvz = dz + 0.5 * cz(q);
        double ubx, uby, ubz;
        surf_vel(A.U, A.W, p, k, A.b.ule, lvx, lvy, lvz, ubx, uby, ubz);
        const int co = opp(q);
        const double ubc = ubx * cx(co) + uby * cy(co) + ubz * cz(co);
        const double corr = 6.0 * wq(co) * A.rho0 * ubc;
        const double fo = (double)Store<ST>::ld(fin, (size_t)co * A.plane + node, co, A.tab);
        n[q] = (CT)(fo - corr);
        // eq. (6): momentum exchanged across the link (deviation form: the rest-state
        // part 2 w rho0 c cancels between the entry and exit links of each line)
        const double fm = 2.0 * fo - corr;
        const double fx = fm * cx(co), fy = fm * cy(co), fz = fm * cz(co);
        if (p != acc.p) {
          if (acc.p >= 0) link_flush_atomic(A.hyd, acc);
          acc.p = p;
#pragma unroll
          for (int c = 0; c < HYD; ++c) acc.v[c] = 0.0;
        }
        acc.v[0] += fx; acc.v[1] += fy; acc.v[2] += fz;
        acc.v[3] += lvy * fz - lvz * fy;
        acc.v[4] += lvz * fx - lvx * fz;
        acc.v[5] += lvx * fy - lvy * fx;
        acc.v[6] += lvx * fx;
        acc.v[7] += lvy * fy;
        acc.v[8] += lvz * fz;
        acc.v[9] += 0.5 * (lvx * fy + lvy * fx);
        acc.v[10] += 0.5 * (lvx * fz + lvz * fx);
        acc.v[11] += 0.5 * (lvy * fz + lvz * fy);
        acc.v[12] += 1.0;
      }
    }
    // eq. (4) moments and BGK collision on the deviations d_q = n_q - w_q rho0
    CT rd = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      rd += n[q];
      jx += n[q] * (CT)cx(q);
      jy += n[q] * (CT)cy(q);
      jz += n[q] * (CT)cz(q);
    }
    const CT rho = (CT)A.rho0 + rd;
    const CT ux = jx / rho, uy = jy / rho, uz = jz / rho;
    const CT uu = ux * ux + uy * uy + uz * uz;
    const CT om = (CT)A.omega;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const CT cu = (CT)cx(q) * ux + (CT)cy(q) * uy + (CT)cz(q) * uz;
      const CT feqd = (CT)wq(q) * (rd + rho * ((CT)3 * cu + (CT)4.5 * cu * cu - (CT)1.5 * uu));
      const CT ne = n[q] - feqd;
      if (cx(q) != 0) pn[0] += ne;
      if (cy(q) != 0) pn[1] += ne;
      if (cz(q) != 0) pn[2] += ne;
      if (cx(q) * cy(q) != 0) pn[3] += ne * (CT)(cx(q) * cy(q));
      if (cx(q) * cz(q) != 0) pn[4] += ne * (CT)(cx(q) * cz(q));
      if (cy(q) * cz(q) != 0) pn[5] += ne * (CT)(cy(q) * cz(q));
      Store<ST>::st(fout, (size_t)q * A.plane + node, n[q] - om * ne, q, A.tab);
    }
  }
  // ---- per-sphere sums of the wave's links: one atomic set per sphere and wave ----
  {
    uint64_t mask = __ballot(acc.p >= 0);
    while (mask) {
      const int leader = __ffsll((unsigned long long)mask) - 1;
      const int p = __shfl(acc.p, leader, 64);
      const bool mine = acc.p == p;
      const uint64_t mm = __ballot(mine);
      double tot[HYD];
#pragma unroll
      for (int c = 0; c < HYD; ++c) tot[c] = wave_sum(mine ? acc.v[c] : 0.0);
      if ((int)(threadIdx.x & 63) == leader) {
#pragma unroll
        for (int c = 0; c < HYD; ++c) unsafeAtomicAdd(&A.hyd[(size_t)p * HYD + c], tot[c]);
      }
      if (mine) acc.p = -1;
      mask &= ~mm;
    }
  }
  // ---- block partial of the non-equilibrium momentum flux (fluid stress) ----
  __shared__ double red[LBM_BLOCK / 64][6];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    double v = wave_sum((double)pn[c]);
    if (lane == 0) red[wv][c] = v;
  }
  __syncthreads();
  if (threadIdx.x < 6 && blk_ok) {
    double v = 0;
    for (int w = 0; w < LBM_BLOCK / 64; ++w) v += red[w][threadIdx.x];
    A.pineq[(size_t)blk * 6 + threadIdx.x] = v;
  }
}

hipError_t launch_lbm(Sim *s, const Box &b) {
  LbmArgs A;
  A.fin = s->f[s->cur];
  A.fout = s->f[1 - s->cur];
  A.plane = s->plane;
  A.own = s->own[s->own_cur];
  A.gown = s->gown;
  A.gval = s->gval;
  A.R = s->R[s->pcur];
  A.U = s->U[s->pcur];
  A.W = s->W[s->pcur];
  A.hyd = s->hyd[s->hcur];
  A.pineq = s->pineq;
  A.nodes = s->nodes;
  A.lx = s->lx; A.ly = s->ly; A.lz = s->lz;
  A.nblk = s->lbm_blocks;
  A.per_xcd = (s->lbm_blocks + 7) / 8;
  A.b = b;
  A.rho0 = s->rho0;
  A.omega = 1.0 / s->tau;
  for (int i = 0; i < 2 * NQ; ++i) A.tab[i] = s->fp16_tab[i];
  dim3 grid(A.per_xcd * 8), blk(LBM_BLOCK);
  if (s->precision == 0) hipLaunchKernelGGL(k_lbm<double>, grid, blk, 0, s->stream, A);
  else if (s->precision == 1) hipLaunchKernelGGL(k_lbm<float>, grid, blk, 0, s->stream, A);
  else hipLaunchKernelGGL(k_lbm<__half>, grid, blk, 0, s->stream, A);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Neighbour cells of a point (primary-box position px,py,pz) under Lees-Edwards: calls
// fn(cell index) once per distinct cell whose spheres can lie within one cell width.
template <class F>
__device__ inline void for_near_cells(const Cells &C, const Box &b, double px, double py,
                                      double pz, F fn) {
  int ccy = (int)floor(py * C.iy);
  ccy = ccy < 0 ? 0 : (ccy >= C.ny ? C.ny - 1 : ccy);
  int ccz = (int)floor(pz * C.iz);
  ccz = ccz < 0 ? 0 : (ccz >= C.nz ? C.nz - 1 : ccz);
  const int zn = C.nz >= 3 ? 3 : C.nz;
  const int xn = C.nx >= 3 ? 3 : C.nx;
  for (int dy = -1; dy <= 1; ++dy) {
    int ny = ccy + dy;
    double xs = px;
    if (ny < 0) { ny += C.ny; xs = px + b.s; }
    else if (ny >= C.ny) { ny -= C.ny; xs = px - b.s; }
    xs = xs - b.Lx * floor(xs / b.Lx);
    int ccx = (int)floor(xs * C.ix);
    ccx = ccx < 0 ? 0 : (ccx >= C.nx ? C.nx - 1 : ccx);
    for (int iz = 0; iz < zn; ++iz) {
      int nz = C.nz >= 3 ? ccz + iz - 1 : iz;
      nz = nz < 0 ? nz + C.nz : (nz >= C.nz ? nz - C.nz : nz);
      for (int ix = 0; ix < xn; ++ix) {
        int nx = C.nx >= 3 ? ccx + ix - 1 : ix;
        nx = nx < 0 ? nx + C.nx : (nx >= C.nx ? nx - C.nx : nx);
        fn(nx + C.nx * (ny + C.ny * nz));
      }
    }
  }
}

struct GhostArgs {
  const void *fin;
  size_t plane;
  const int32_t *own;
  const double *R, *U, *W, *amap;
  const int32_t *cell_start, *cell_ids;
  Cells C;
  Box b;
  int lx, ly, lz, n;
  double rho0;
  int values;
  int32_t *gown;
  void *gval;
  int32_t *flags;
  float tab[2 * NQ];
};

// Galilean-corrected post-collision deviation of direction q at node (x,yrow,z) seen from
// the neighbouring image box: sgn = +1 box below (u - ule), -1 box above (u + ule).
template <class ST, class CT>
__device__ inline CT nhat(const GhostArgs &A, const ST *fin, int q, int x, int yrow, int z,
                          int sgn) {
  const int64_t node = x + (int64_t)A.lx * (yrow + (int64_t)A.ly * z);
  const int o = A.own[node];
  if (o >= 0) {
    double dx, dy, dz;
    int k;
    minimage(A.b, (double)x - A.R[3 * o], (double)yrow - A.R[3 * o + 1],
             (double)z - A.R[3 * o + 2], dx, dy, dz, k);
    double ux, uy, uz;
    surf_vel(A.U, A.W, o, k, A.b.ule, dx, dy, dz, ux, uy, uz);
    ux -= sgn * A.b.ule;
    const double cu = cx(q) * ux + cy(q) * uy + cz(q) * uz;
    const double uu = ux * ux + uy * uy + uz * uz;
    return (CT)(wq(q) * A.rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
  }
  CT rd = 0, jx = 0, jy = 0, jz = 0, fq = 0;
#pragma unroll
  for (int r = 0; r < NQ; ++r) {
    const CT v = Store<ST>::ld(fin, (size_t)r * A.plane + node, r, A.tab);
    rd += v; jx += v * (CT)cx(r); jy += v * (CT)cy(r); jz += v * (CT)cz(r);
    if (r == q) fq = v;
  }
  const CT rho = (CT)A.rho0 + rd;
  const CT ux = jx / rho, uy = jy / rho, uz = jz / rho;
  // feq(rho, u + du) - feq(rho, u) with du = -sgn ule x, written out to avoid cancellation
  const CT du = (CT)(-sgn * A.b.ule);
  const CT cu = (CT)cx(q) * ux + (CT)cy(q) * uy + (CT)cz(q) * uz;
  const CT cd = (CT)cx(q) * du;
  const CT dfe = (CT)wq(q) * rho * ((CT)3 * cd + (CT)4.5 * cd * ((CT)2 * cu + cd) -
                                    (CT)1.5 * du * ((CT)2 * ux + du));
  return fq + dfe;
}

template <class ST>
__global__ void k_ghosts(GhostArgs A) {
  using CT = typename Store<ST>::CT;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int npl = A.lx * A.lz;
  if (idx >= 2 * npl) return;
  const int g = idx / npl;
  const int rem = idx - g * npl;
  const int z = rem / A.lx, x = rem - (rem / A.lx) * A.lx;
  const double gy = g == 0 ? -1.0 : (double)A.ly;
  // primary-box position of the ghost point, for the cell search only
  double px = g == 0 ? (double)x + A.b.s : (double)x - A.b.s;
  px = px - A.b.Lx * floor(px / A.b.Lx);
  const double py = g == 0 ? (double)(A.ly - 1) : 0.0;
  int owner = -1, clash = 0;
  if (A.n > 0) for_near_cells(A.C, A.b, px, py, (double)z, [&](int c) {
    for (int t = A.cell_start[c]; t < A.cell_start[c + 1]; ++t) {
      const int p = A.cell_ids[t];
      double dx, dy, dz;
      int k;
      minimage(A.b, (double)x - A.R[3 * p], gy - A.R[3 * p + 1], (double)z - A.R[3 * p + 2],
               dx, dy, dz, k);
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (r2 < A.amap[p] * A.amap[p]) {
        if (owner >= 0 && owner != p) clash = 1;
        if (owner < 0 || p < owner) owner = p;
      }
    }
  });
  if (clash) atomicOr(A.flags, 1);
  A.gown[idx] = owner;
  if (!A.values || owner >= 0) return;
  const ST *fin = (const ST *)A.fin;
  CT *gval = (CT *)A.gval;
  const int sgn = g == 0 ? 1 : -1;
  const int yrow = g == 0 ? A.ly - 1 : 0;
  const double xs = (double)x + sgn * A.b.s;
  const double x0f = floor(xs);
  const double fr = xs - x0f;
  int i0 = (int)x0f % A.lx;
  i0 = i0 < 0 ? i0 + A.lx : i0;
  const int i1 = i0 + 1 == A.lx ? 0 : i0 + 1;
  for (int m = 0; m < 5; ++m) {
    const int q = gdir(g, m);
    const CT v0 = nhat<ST, CT>(A, fin, q, i0, yrow, z, sgn);
    const CT v1 = nhat<ST, CT>(A, fin, q, i1, yrow, z, sgn);
    gval[(size_t)((g * 5 + m) * A.lz + z) * A.lx + x] = ((CT)1 - (CT)fr) * v0 + (CT)fr * v1;
  }
}

hipError_t launch_ghosts(Sim *s, const Box &b, int32_t *gown_out, void *gval_out, int values) {
  GhostArgs A;
  A.fin = s->f[s->cur];
  A.plane = s->plane;
  A.own = s->own[s->own_cur];
  A.R = s->R[s->pcur]; A.U = s->U[s->pcur]; A.W = s->W[s->pcur];
  A.amap = s->amap;
  A.cell_start = s->cell_start;
  A.cell_ids = s->cell_ids;
  A.C = s->cells;
  A.b = b;
  A.lx = s->lx; A.ly = s->ly; A.lz = s->lz; A.n = s->n;
  A.rho0 = s->rho0;
  A.values = values;
  A.gown = gown_out;
  A.gval = gval_out;
  A.flags = s->flags;
  for (int i = 0; i < 2 * NQ; ++i) A.tab[i] = s->fp16_tab[i];
  const int tot = 2 * s->lx * s->lz;
  dim3 grid((tot + 255) / 256), blk(256);
  if (s->precision == 0) hipLaunchKernelGGL(k_ghosts<double>, grid, blk, 0, s->stream, A);
  else if (s->precision == 1) hipLaunchKernelGGL(k_ghosts<float>, grid, blk, 0, s->stream, A);
  else hipLaunchKernelGGL(k_ghosts<__half>, grid, blk, 0, s->stream, A);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
struct Tab {
  float v[2 * NQ];
};

// Equilibrium of the imposed linear shear profile u_x = gd (y - (ly-1)/2) at rho0.
template <class ST>
__global__ void k_init_pop(void *fv, size_t plane, int64_t nodes, int lx, int ly, double gd,
                           double rho0, Tab tab) {
  using CT = typename Store<ST>::CT;
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= nodes) return;
  ST *f = (ST *)fv;
  const int y = (int)((node / lx) % ly);
  const double ux = gd * ((double)y - 0.5 * (double)(ly - 1));
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double cu = cx(q) * ux;
    const double d = wq(q) * rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * ux * ux);
    Store<ST>::st(f, (size_t)q * plane + node, (CT)d, q, tab.v);
  }
}

// FP64 full populations <-> storage deviations.
template <class ST>
__global__ void k_pop_convert(void *fv, double *d64, size_t plane, int64_t nodes, double rho0,
                              int to_storage, Tab tab) {
  using CT = typename Store<ST>::CT;
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= nodes) return;
  ST *f = (ST *)fv;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double w = wq(q) * rho0;
    if (to_storage)
      Store<ST>::st(f, (size_t)q * plane + node, (CT)(d64[(size_t)q * nodes + node] - w), q, tab.v);
    else
      d64[(size_t)q * nodes + node] = w + (double)Store<ST>::ld(f, (size_t)q * plane + node, q, tab.v);
  }
}

static Tab make_tab(const Sim *s) {
  Tab t;
  for (int i = 0; i < 2 * NQ; ++i) t.v[i] = s->fp16_tab[i];
  return t;
}

hipError_t launch_init_populations(Sim *s) {
  double gd = 0.0;
  // gdot(0): simple shear rate, or omega g0_I sin(Theta) for eq. (16)
  if (s->shear_kind == 1) gd = s->gamma_dot;
  else if (s->shear_kind == 2) {
    const double om = 2.0 * 3.14159265358979323846 / (double)s->period;
    gd = om * s->g0_I * sin(s->theta);
  }
  dim3 grid((unsigned)((s->nodes + 255) / 256)), blk(256);
  for (int b = 0; b < 2; ++b) {
    if (s->precision == 0)
      hipLaunchKernelGGL(k_init_pop<double>, grid, blk, 0, s->stream, s->f[b], s->plane, s->nodes, s->lx, s->ly, gd, s->rho0, make_tab(s));
    else if (s->precision == 1)
      hipLaunchKernelGGL(k_init_pop<float>, grid, blk, 0, s->stream, s->f[b], s->plane, s->nodes, s->lx, s->ly, gd, s->rho0, make_tab(s));
    else
      hipLaunchKernelGGL(k_init_pop<__half>, grid, blk, 0, s->stream, s->f[b], s->plane, s->nodes, s->lx, s->ly, gd, s->rho0, make_tab(s));
  }
  return hipGetLastError();
}

hipError_t launch_pop_convert(Sim *s, double *dev64, int to_storage) {
  dim3 grid((unsigned)((s->nodes + 255) / 256)), blk(256);
  void *f = s->f[s->cur];
  if (s->precision == 0)
    hipLaunchKernelGGL(k_pop_convert<double>, grid, blk, 0, s->stream, f, dev64, s->plane, s->nodes, s->rho0, to_storage, make_tab(s));
  else if (s->precision == 1)
    hipLaunchKernelGGL(k_pop_convert<float>, grid, blk, 0, s->stream, f, dev64, s->plane, s->nodes, s->rho0, to_storage, make_tab(s));
  else
    hipLaunchKernelGGL(k_pop_convert<__half>, grid, blk, 0, s->stream, f, dev64, s->plane, s->nodes, s->rho0, to_storage, make_tab(s));
  return hipGetLastError();
}

// Every (node, q) whose pull source x - c_q is solid (map or ghost plane): owner, else -1.
__global__ void k_link_enum(const int32_t *own, const int32_t *gown, int64_t nodes, int lx,
                            int ly, int lz, int32_t *out) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= nodes) return;
  const bool fluid = own[node] == -1;
  const int x = (int)(node % lx);
  const int64_t yz = node / lx;
  const int y = (int)(yz % ly), z = (int)(yz / ly);
  out[node] = -1;
  for (int q = 1; q < NQ; ++q) {
    int so = -1;
    if (fluid) {
      int px = x - cx(q), py = y - cy(q), pz = z - cz(q);
      px = px < 0 ? px + lx : (px >= lx ? px - lx : px);
      pz = pz < 0 ? pz + lz : (pz >= lz ? pz - lz : pz);
      if (py < 0 || py >= ly) so = gown[((py < 0 ? 0 : 1) * lz + pz) * lx + px];
      else so = own[px + (int64_t)lx * (py + (int64_t)ly * pz)];
      if (so < 0) so = -1;
    }
    out[(size_t)q * nodes + node] = so;
  }
}

hipError_t launch_link_enum(Sim *s, const int32_t *gown, int32_t *out, const Box &b) {
  (void)b;
  dim3 grid((unsigned)((s->nodes + 255) / 256)), blk(256);
  hipLaunchKernelGGL(k_link_enum, grid, blk, 0, s->stream, s->own[s->own_cur], gown, s->nodes,
                     s->lx, s->ly, s->lz, out);
  return hipGetLastError();
}

}  // namespace susp
