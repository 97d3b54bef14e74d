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
// Fused lattice kernel.
//
// A work-group owns one brick of TX x BY x BZ nodes and walks it in tiles of TX x TY
// (one wave per 64-node row segment).  Per tile the owner map with a one-node halo is
// staged in LDS (halo rows outside the box come from the Lees-Edwards ghost planes), so
// every pull source is classified from LDS.
//
// Links: with lever r_b - R = D - c_q/2 (D = node minus sphere centre, minimum image) the
// surface velocity along the link is u_b.c_q = u(X).c_q, because (W x c).c = 0; hence one
// FP64 minimum image and one rigid-body velocity per node and sphere, and per link only
//   corr = -6 w_q rho0 u(X).c_q,  n_q = n*_qbar - corr,  m = 2 n*_qbar - corr.
// The node's sums are F = -sum m c_q, T = D x F, S = sym(D (x) F) + 1/2 sum m c_q c_q
// (exactly the link sums of eqs. 6, 9, 10 regrouped).  Per-sphere sums of the brick are
// accumulated in an LDS hash table (two copies to halve atomic contention) and written
// once per brick; k_hydro_gather adds a sphere's brick entries in a fixed order.
constexpr int TX = 64, TY = 4;
constexpr int TSLOT = 128;

struct LbmArgs {
  const void *fin;
  void *fout;
  size_t plane;
  const int32_t *own;
  const int32_t *gown;
  const void *gval;
  const double *R, *U, *W;
  int32_t *bt_key;
  double *bt_val;
  double *hyd_fb;
  double *pineq;
  int32_t *flags;
  int lx, ly, lz;
  int bxn, byn, bzn, BY, BZ;
  int nbricks, per_xcd;
  Box b;
  double rho0, omega;
  H16 h16;
};

// Slot of sphere p in a brick's LDS table (open addressing), or -1 if the table is full.
__device__ inline int table_slot(int32_t *skey, int p) {
  int h = p & (TSLOT - 1);
  for (int probe = 0; probe < TSLOT; ++probe) {
    int key = skey[h];
    if (key == -1) key = atomicCAS(&skey[h], -1, p);
    if (key == -1 || key == p) return h;
    h = (h + 1) & (TSLOT - 1);
  }
  return -1;
}

template <class ST>
__global__ __launch_bounds__(256, 3) void k_lbm(LbmArgs A) {
  using CT = typename Store<ST>::CT;
  const ST *fin = (const ST *)A.fin;
  ST *fout = (ST *)A.fout;
  const CT *gval = (const CT *)A.gval;
  __shared__ int32_t smap[3][TY + 2][TX + 2];
  __shared__ int32_t skey[TSLOT];
  __shared__ double sval[2][TSLOT][HYD];
  __shared__ double red[4][6];
  // XCD-aware brick order: hardware blocks are dealt round-robin to the 8 XCDs; each XCD
  // gets a contiguous range of bricks (z-major), so neighbouring bricks share its L2
  const int hb = blockIdx.x;
  int brick = (hb & 7) * A.per_xcd + (hb >> 3);
  const bool bok = brick < A.nbricks;
  if (!bok) brick = 0;
  const int bxi = brick % A.bxn;
  const int byi = (brick / A.bxn) % A.byn;
  const int bzi = brick / (A.bxn * A.byn);
  const int t = threadIdx.x;
  const int tx = t & 63, tyl = t >> 6;
  const int lx = A.lx, ly = A.ly, lz = A.lz;
  for (int i = t; i < TSLOT; i += 256) skey[i] = -1;
  for (int i = t; i < 2 * TSLOT * HYD; i += 256) (&sval[0][0][0])[i] = 0.0;
  double pn[6] = {0, 0, 0, 0, 0, 0};
  const int x0 = bxi * TX;
  const int x = x0 + tx;
  const int z_end = min(lz, (bzi + 1) * A.BZ), y_end = min(ly, (byi + 1) * A.BY);
  for (int z = bzi * A.BZ; bok && z < z_end; ++z) {
    for (int y0 = byi * A.BY; y0 < y_end; y0 += TY) {
      __syncthreads();  // previous tile done with smap (and table initialised)
      for (int i = t; i < 3 * (TY + 2) * (TX + 2); i += 256) {
        const int dx = i % (TX + 2), dy = (i / (TX + 2)) % (TY + 2), dz = i / ((TX + 2) * (TY + 2));
        int gx = (x0 - 1 + dx) % lx;
        gx = gx < 0 ? gx + lx : gx;
        int gz = (z - 1 + dz) % lz;
        gz = gz < 0 ? gz + lz : gz;
        const int gy = y0 - 1 + dy;
        int v;
        if (gy < 0) v = A.gown[(0 * lz + gz) * lx + gx];
        else if (gy >= ly) v = A.gown[(1 * lz + gz) * lx + gx];
        else v = A.own[gx + (int64_t)lx * (gy + (int64_t)ly * gz)];
        smap[dz][dy][dx] = v;
      }
      __syncthreads();
      const int y = y0 + tyl;
      const bool valid = x < lx && y < ly;
      const int own = valid ? smap[1][tyl + 1][tx + 1] : -2;
      if (own == -2) continue;
      const int node = x + lx * (y + ly * z);  // < 2^31 nodes (checked at creation)
      if (own >= 0) {
        // solid node: its populations are never read (a released node is refilled); store
        // the rest state so that the wave writes whole cache lines
#pragma unroll
        for (int q = 0; q < NQ; ++q) Store<ST>::st(fout + (size_t)q * A.plane, node, (CT)0, q, A.h16);
        continue;
      }
      CT n[NQ];
      uint32_t lmask = 0, m2 = 0;  // links; links to a sphere other than p1
      int p1 = -1;
      n[0] = Store<ST>::ld(fin, node, 0, A.h16);
#pragma unroll
      for (int q = 1; q < NQ; ++q) {
        const int so = smap[1 - cz(q)][tyl + 1 - cy(q)][tx + 1 - cx(q)];
        if (so >= 0) {
          if (p1 < 0) p1 = so;
          else if (so != p1) m2 |= 1u << q;
        }
        // exactly one independent load per direction: the pulled population if the
        // source is fluid, else this node's own opposite population (bounced back below)
        CT val;
        if (so < 0) {
          int px = x - cx(q), pz = z - cz(q);
          const int py = y - cy(q);
          px = px < 0 ? px + lx : (px >= lx ? px - lx : px);
          pz = pz < 0 ? pz + lz : (pz >= lz ? pz - lz : pz);
          if (cy(q) != 0 && (py < 0 || py >= ly))
            val = gval[((((py < 0 ? 0 : 1) * 5 + gslot(q)) * lz + pz) * lx + px)];
          else
            val = Store<ST>::ld(fin + (size_t)q * A.plane, px + lx * (py + ly * pz), q, A.h16);
        } else {
          lmask |= 1u << q;
          val = Store<ST>::ld(fin + (size_t)opp(q) * A.plane, node, opp(q), A.h16);
        }
        n[q] = val;
      }
      // ---- links, one sphere at a time (a node rarely touches more than two) ----
      for (int it = 0; it < 6 && lmask; ++it) {
        // first pass: sphere p1 (links lmask & ~m2, no map reads); later passes: the
        // sphere of the lowest remaining link
        int p = p1;
        uint32_t mine = lmask & ~m2;
        if (it > 0) {
          p = -1;
#pragma unroll
          for (int q = NQ - 1; q >= 1; --q)
            if ((lmask >> q) & 1u) p = smap[1 - cz(q)][tyl + 1 - cy(q)][tx + 1 - cx(q)];
          mine = 0;
#pragma unroll
          for (int q = 1; q < NQ; ++q)
            if (((lmask >> q) & 1u) && smap[1 - cz(q)][tyl + 1 - cy(q)][tx + 1 - cx(q)] == p) mine |= 1u << q;
        }
        double Dx, Dy, Dz;
        int k;
        minimage(A.b, (double)x - A.R[3 * p], (double)y - A.R[3 * p + 1], (double)z - A.R[3 * p + 2],
                 Dx, Dy, Dz, k);
        const double w0 = A.W[3 * p], w1 = A.W[3 * p + 1], w2 = A.W[3 * p + 2];
        const double U0 = A.U[3 * p], U1 = A.U[3 * p + 1], U2 = A.U[3 * p + 2];
        const int slot = table_slot(skey, p);
        double *dst = slot >= 0 ? &sval[t & 1][slot][0] : &A.hyd_fb[(size_t)p * HYD];
        // every link source X - c_q lies in the image of X itself unless X is within one
        // node of half a period from the centre (thin boxes); then each link finds its own
        const bool same_image = fabs(Dx) <= 0.5 * A.b.Lx - 1.000001 &&
                                fabs(Dy) <= 0.5 * A.b.Ly - 1.000001 &&
                                fabs(Dz) <= 0.5 * A.b.Lz - 1.000001;
        if (same_image) {
          const double ux = U0 + k * A.b.ule + (w1 * Dz - w2 * Dy);
          const double uy = U1 + (w2 * Dx - w0 * Dz);
          const double uz = U2 + (w0 * Dy - w1 * Dx);
          double g0 = 0, g1 = 0, g2 = 0, mxx = 0, myy = 0, mzz = 0, mxy = 0, mxz = 0, myz = 0, cnt = 0;
#pragma unroll
          for (int q = 1; q < NQ; ++q) {
            if ((mine >> q) & 1u) {
              const double fo = (double)n[q];
              const double ucq = cx(q) * ux + cy(q) * uy + cz(q) * uz;
              const double corr = -6.0 * wq(q) * A.rho0 * ucq;
              n[q] = (CT)(fo - corr);
              const double m = 2.0 * fo - corr;
              g0 += cx(q) * m; g1 += cy(q) * m; g2 += cz(q) * m;
              mxx += cx(q) * cx(q) * m; myy += cy(q) * cy(q) * m; mzz += cz(q) * cz(q) * m;
              mxy += cx(q) * cy(q) * m; mxz += cx(q) * cz(q) * m; myz += cy(q) * cz(q) * m;
              cnt += 1.0;
            }
          }
          double v[HYD];
          v[0] = -g0; v[1] = -g1; v[2] = -g2;
          v[3] = Dy * v[2] - Dz * v[1];
          v[4] = Dz * v[0] - Dx * v[2];
          v[5] = Dx * v[1] - Dy * v[0];
          v[6] = Dx * v[0] + 0.5 * mxx;
          v[7] = Dy * v[1] + 0.5 * myy;
          v[8] = Dz * v[2] + 0.5 * mzz;
          v[9] = 0.5 * (Dx * v[1] + Dy * v[0]) + 0.5 * mxy;
          v[10] = 0.5 * (Dx * v[2] + Dz * v[0]) + 0.5 * mxz;
          v[11] = 0.5 * (Dy * v[2] + Dz * v[1]) + 0.5 * myz;
          v[12] = cnt;
#pragma unroll
          for (int c = 0; c < HYD; ++c) unsafeAtomicAdd(&dst[c], v[c]);
        } else {
#pragma unroll
          for (int q = 1; q < NQ; ++q) {
            if ((mine >> q) & 1u) {
              // lever of this link from the image that holds its solid end (eq. 8)
              double ex, ey, ez;
              int kq;
              minimage(A.b, (double)(x - cx(q)) - A.R[3 * p], (double)(y - cy(q)) - A.R[3 * p + 1],
                       (double)(z - cz(q)) - A.R[3 * p + 2], ex, ey, ez, kq);
              const double lvx = ex + 0.5 * cx(q), lvy = ey + 0.5 * cy(q), lvz = ez + 0.5 * cz(q);
              const double ubx = U0 + kq * A.b.ule + (w1 * lvz - w2 * lvy);
              const double uby = U1 + (w2 * lvx - w0 * lvz);
              const double ubz = U2 + (w0 * lvy - w1 * lvx);
              const double fo = (double)n[q];
              const double corr = -6.0 * wq(q) * A.rho0 * (cx(q) * ubx + cy(q) * uby + cz(q) * ubz);
              n[q] = (CT)(fo - corr);
              const double m = 2.0 * fo - corr;
              const double fx = -cx(q) * m, fy = -cy(q) * m, fz = -cz(q) * m;
              double v[HYD];
              v[0] = fx; v[1] = fy; v[2] = fz;
              v[3] = lvy * fz - lvz * fy;
              v[4] = lvz * fx - lvx * fz;
              v[5] = lvx * fy - lvy * fx;
              v[6] = lvx * fx; v[7] = lvy * fy; v[8] = lvz * fz;
              v[9] = 0.5 * (lvx * fy + lvy * fx);
              v[10] = 0.5 * (lvx * fz + lvz * fx);
              v[11] = 0.5 * (lvy * fz + lvz * fy);
              v[12] = 1.0;
#pragma unroll
              for (int c = 0; c < HYD; ++c) unsafeAtomicAdd(&dst[c], v[c]);
            }
          }
        }
        lmask &= ~mine;
      }
      if (lmask) atomicOr(A.flags, 8);
      // ---- eq. (4) moments and BGK collision on the deviations d_q = n_q - w_q rho0 ----
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
      CT s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const CT cu = (CT)cx(q) * ux + (CT)cy(q) * uy + (CT)cz(q) * uz;
        const CT feqd = (CT)wq(q) * (rd + rho * ((CT)3 * cu + (CT)4.5 * cu * cu - (CT)1.5 * uu));
        const CT ne = n[q] - feqd;
        if (cx(q) != 0) s0 += ne;
        if (cy(q) != 0) s1 += ne;
        if (cz(q) != 0) s2 += ne;
        if (cx(q) * cy(q) != 0) s3 += ne * (CT)(cx(q) * cy(q));
        if (cx(q) * cz(q) != 0) s4 += ne * (CT)(cx(q) * cz(q));
        if (cy(q) * cz(q) != 0) s5 += ne * (CT)(cy(q) * cz(q));
        Store<ST>::st(fout + (size_t)q * A.plane, node, n[q] - om * ne, q, A.h16);
      }
      pn[0] += (double)s0; pn[1] += (double)s1; pn[2] += (double)s2;
      pn[3] += (double)s3; pn[4] += (double)s4; pn[5] += (double)s5;
    }
  }
  __syncthreads();
  // ---- brick table out ----
  if (bok)
    for (int i = t; i < TSLOT; i += 256) {
      const int key = skey[i];
      A.bt_key[(size_t)brick * TSLOT + i] = key;
      if (key >= 0)
        for (int c = 0; c < HYD; ++c)
          A.bt_val[((size_t)brick * TSLOT + i) * HYD + c] = sval[0][i][c] + sval[1][i][c];
    }
  // ---- brick partial of the non-equilibrium momentum flux (fluid stress) ----
  const int lane = t & 63, wv = t >> 6;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    double v = wave_sum(pn[c]);
    if (lane == 0) red[wv][c] = v;
  }
  __syncthreads();
  if (t < 6 && bok) A.pineq[(size_t)brick * 6 + t] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
}

hipError_t launch_lbm(Sim *s, const Box &b) {
  LbmArgs A;
  A.fin = s->f[s->cur];
  A.fout = s->f[1 - s->cur];
  A.plane = s->plane;
  A.own = s->own;
  A.gown = s->gown;
  A.gval = s->gval;
  A.R = s->R[s->pcur];
  A.U = s->U[s->pcur];
  A.W = s->W[s->pcur];
  A.bt_key = s->bt_key;
  A.bt_val = s->bt_val;
  A.hyd_fb = s->hyd_fb;
  A.pineq = s->pineq;
  A.flags = s->flags;
  A.lx = s->lx; A.ly = s->ly; A.lz = s->lz;
  A.bxn = s->bxn; A.byn = s->byn; A.bzn = s->bzn; A.BY = s->BY; A.BZ = s->BZ;
  A.nbricks = s->nbricks;
  A.per_xcd = (s->nbricks + 7) / 8;
  A.b = b;
  A.rho0 = s->rho0;
  A.omega = 1.0 / s->tau;
  A.h16 = s->h16;
  dim3 grid(A.per_xcd * 8), blk(256);
  if (s->precision == 0) hipLaunchKernelGGL(k_lbm<double>, grid, blk, 0, s->stream, A);
  else if (s->precision == 1) hipLaunchKernelGGL(k_lbm<float>, grid, blk, 0, s->stream, A);
  else hipLaunchKernelGGL(k_lbm<__half>, grid, blk, 0, s->stream, A);
  return hipGetLastError();
}

// Per-sphere hydrodynamic sums: the entries of every brick the sphere's links can reach
// (nodes within a_map + 2 of any of its Lees-Edwards images), added in brick order, plus
// the overflow accumulator (which is cleared for the next step).  One wave per sphere.
struct GatherArgs {
  const double *R, *amap;
  const int32_t *bt_key;
  const double *bt_val;
  double *hyd_fb;
  double *hyd;
  int n, lx, ly, lz, bxn, byn, BY, BZ;
  double s;
};

// Next node coordinate (along a periodic axis of length L with bricks of B nodes) that
// starts a new brick after coordinate xx.
__device__ inline int next_brick_start(int xx, int L, int B) {
  int w = xx % L;
  w = w < 0 ? w + L : w;
  return xx + (B - (w % B));
}
__device__ inline int brick_of(int xx, int L, int B) {
  int w = xx % L;
  w = w < 0 ? w + L : w;
  return w / B;
}

__global__ __launch_bounds__(256) void k_hydro_gather(GatherArgs A) {
  __shared__ int vis[4][256];
  const int wv = threadIdx.x >> 6;
  const int p = blockIdx.x * 4 + wv;
  const int lane = threadIdx.x & 63;
  if (p >= A.n) return;  // uniform per wave
  const double r = A.amap[p] + 2.0;
  double acc[HYD];
#pragma unroll
  for (int c = 0; c < HYD; ++c) acc[c] = 0.0;
  int nvis = 0;
  int zlo = (int)floor(A.R[3 * p + 2] - r), zhi = (int)ceil(A.R[3 * p + 2] + r);
  if (zhi - zlo + 1 >= A.lz) { zlo = 0; zhi = A.lz - 1; }
  for (int k = -1; k <= 1; ++k) {
    const double cy_ = A.R[3 * p + 1] + k * (double)A.ly;
    int ylo = (int)floor(cy_ - r), yhi = (int)ceil(cy_ + r);
    if (ylo < 0) ylo = 0;
    if (yhi > A.ly - 1) yhi = A.ly - 1;
    if (ylo > yhi) continue;
    const double cx_ = A.R[3 * p] + k * A.s;
    int xlo = (int)floor(cx_ - r), xhi = (int)ceil(cx_ + r);
    if (xhi - xlo + 1 >= A.lx) { xlo = 0; xhi = A.lx - 1; }
    for (int zz = zlo; zz <= zhi; zz = next_brick_start(zz, A.lz, A.BZ)) {
      const int bz = brick_of(zz, A.lz, A.BZ);
      for (int by = ylo / A.BY; by <= yhi / A.BY; ++by) {
        for (int xx = xlo; xx <= xhi; xx = next_brick_start(xx, A.lx, TX)) {
          const int brick = brick_of(xx, A.lx, TX) + A.bxn * (by + A.byn * bz);
          // skip bricks already visited (a wrapped range can reach a brick twice)
          bool dup = false;
          for (int base = 0; base < nvis; base += 64) {
            const int v = base + lane < nvis ? vis[wv][base + lane] : -1;
            if (__ballot(v == brick)) { dup = true; break; }
          }
          if (dup) continue;
          if (nvis < 256) {
            if (lane == 0) vis[wv][nvis] = brick;
            ++nvis;
            __builtin_amdgcn_wave_barrier();
          }
          // find p among the brick's keys (at most one slot holds it)
          int hit = -1;
          for (int s0 = 0; s0 < TSLOT; s0 += 64) {
            const int key = A.bt_key[(size_t)brick * TSLOT + s0 + lane];
            const uint64_t m = __ballot(key == p);
            if (m) { hit = s0 + __ffsll((unsigned long long)m) - 1; break; }
          }
          if (hit >= 0) {
#pragma unroll
            for (int c = 0; c < HYD; ++c) acc[c] += A.bt_val[((size_t)brick * TSLOT + hit) * HYD + c];
          }
        }
      }
    }
  }
  if (lane == 0) {
    for (int c = 0; c < HYD; ++c) {
      A.hyd[(size_t)p * HYD + c] = acc[c] + A.hyd_fb[(size_t)p * HYD + c];
      A.hyd_fb[(size_t)p * HYD + c] = 0.0;
    }
  }
}

hipError_t launch_hydro_gather(Sim *s, const Box &b) {
  GatherArgs A;
  A.R = s->R[s->pcur]; A.amap = s->amap;
  A.bt_key = s->bt_key; A.bt_val = s->bt_val; A.hyd_fb = s->hyd_fb;
  A.hyd = s->hyd[s->hcur];
  A.n = s->n; A.lx = s->lx; A.ly = s->ly; A.lz = s->lz;
  A.bxn = s->bxn; A.byn = s->byn; A.BY = s->BY; A.BZ = s->BZ;
  A.s = b.s;
  if (s->n > 0)
    hipLaunchKernelGGL(k_hydro_gather, dim3((s->n + 3) / 4), dim3(256), 0, s->stream, A);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
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
  H16 h16;
};

// Galilean-corrected post-collision deviation of direction q at node (x,yrow,z) seen from
// the neighbouring image box: sgn = +1 box below (u - ule), -1 box above (u + ule).
template <class ST, class CT>
__device__ inline CT nhat(const ST *fin, size_t plane, const int32_t *own, const double *R,
                          const double *U, const double *W, Box b, double rho0, H16 h16, int q,
                          int x, int yrow, int z, int sgn) {
  const int64_t node = x + (int64_t)b.lx * (yrow + (int64_t)b.ly * z);
  const int o = own[node];
  if (o >= 0) {
    double dx, dy, dz;
    int k;
    minimage(b, (double)x - R[3 * o], (double)yrow - R[3 * o + 1], (double)z - R[3 * o + 2], dx, dy,
             dz, k);
    double ux, uy, uz;
    surf_vel(U, W, o, k, b.ule, dx, dy, dz, ux, uy, uz);
    ux -= sgn * b.ule;
    const double cu = cx(q) * ux + cy(q) * uy + cz(q) * uz;
    const double uu = ux * ux + uy * uy + uz * uz;
    return (CT)(wq(q) * rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
  }
  CT rd = 0, jx = 0, jy = 0, jz = 0, fq = 0;
#pragma unroll
  for (int r = 0; r < NQ; ++r) {
    const CT v = Store<ST>::ld(fin, (size_t)r * plane + node, r, h16);
    rd += v; jx += v * (CT)cx(r); jy += v * (CT)cy(r); jz += v * (CT)cz(r);
    if (r == q) fq = v;
  }
  const CT rho = (CT)rho0 + rd;
  const CT ux = jx / rho, uy = jy / rho, uz = jz / rho;
  // feq(rho, u + du) - feq(rho, u) with du = -sgn ule x, written out to avoid cancellation
  const CT du = (CT)(-sgn * b.ule);
  const CT cu = (CT)cx(q) * ux + (CT)cy(q) * uy + (CT)cz(q) * uz;
  const CT cd = (CT)cx(q) * du;
  const CT dfe = (CT)wq(q) * rho * ((CT)3 * cd + (CT)4.5 * cd * ((CT)2 * cu + cd) -
                                    (CT)1.5 * du * ((CT)2 * ux + du));
  return fq + dfe;
}

template <class ST>
__global__ __launch_bounds__(256) void k_ghosts(GhostArgs A) {
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
  if (A.n > 0) {
    const Cells &C = A.C;
    int ccy = (int)floor(py * C.iy);
    ccy = ccy < 0 ? 0 : (ccy >= C.ny ? C.ny - 1 : ccy);
    int ccz = (int)floor((double)z * C.iz);
    ccz = ccz < 0 ? 0 : (ccz >= C.nz ? C.nz - 1 : ccz);
    const int zn = C.nz >= 3 ? 3 : C.nz, xn = C.nx >= 3 ? 3 : C.nx;
    for (int dy = -1; dy <= 1; ++dy) {
      int ny = ccy + dy;
      double xs = px;
      if (ny < 0) { ny += C.ny; xs = px + A.b.s; }
      else if (ny >= C.ny) { ny -= C.ny; xs = px - A.b.s; }
      xs = xs - A.b.Lx * floor(xs / A.b.Lx);
      int ccx = (int)floor(xs * C.ix);
      ccx = ccx < 0 ? 0 : (ccx >= C.nx ? C.nx - 1 : ccx);
      for (int iz = 0; iz < zn; ++iz) {
        int nz = C.nz >= 3 ? ccz + iz - 1 : iz;
        nz = nz < 0 ? nz + C.nz : (nz >= C.nz ? nz - C.nz : nz);
        for (int ix = 0; ix < xn; ++ix) {
          int nx = C.nx >= 3 ? ccx + ix - 1 : ix;
          nx = nx < 0 ? nx + C.nx : (nx >= C.nx ? nx - C.nx : nx);
          const int c = nx + C.nx * (ny + C.ny * nz);
          for (int t = A.cell_start[c]; t < A.cell_start[c + 1]; ++t) {
            const int p = A.cell_ids[t];
            double dx, dy2, dz;
            int k;
            minimage(A.b, (double)x - A.R[3 * p], gy - A.R[3 * p + 1], (double)z - A.R[3 * p + 2],
                     dx, dy2, dz, k);
            const double r2 = dx * dx + dy2 * dy2 + dz * dz;
            if (r2 < A.amap[p] * A.amap[p]) {
              if (owner >= 0 && owner != p) clash = 1;
              if (owner < 0 || p < owner) owner = p;
            }
          }
        }
      }
    }
  }
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
    const CT v0 = nhat<ST, CT>(fin, A.plane, A.own, A.R, A.U, A.W, A.b, A.rho0, A.h16, q, i0, yrow, z, sgn);
    const CT v1 = nhat<ST, CT>(fin, A.plane, A.own, A.R, A.U, A.W, A.b, A.rho0, A.h16, q, i1, yrow, z, sgn);
    gval[(size_t)((g * 5 + m) * A.lz + z) * A.lx + x] = ((CT)1 - (CT)fr) * v0 + (CT)fr * v1;
  }
}

hipError_t launch_ghosts(Sim *s, const Box &b, int32_t *gown_out, void *gval_out, int values) {
  GhostArgs A;
  A.fin = s->f[s->cur];
  A.plane = s->plane;
  A.own = s->own;
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
  A.h16 = s->h16;
  const int tot = 2 * s->lx * s->lz;
  dim3 grid((tot + 255) / 256), blk(256);
  if (s->precision == 0) hipLaunchKernelGGL(k_ghosts<double>, grid, blk, 0, s->stream, A);
  else if (s->precision == 1) hipLaunchKernelGGL(k_ghosts<float>, grid, blk, 0, s->stream, A);
  else hipLaunchKernelGGL(k_ghosts<__half>, grid, blk, 0, s->stream, A);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Equilibrium of the imposed linear shear profile u_x = gd (y - (ly-1)/2) at rho0.
template <class ST>
__global__ void k_init_pop(void *fv, size_t plane, int64_t nodes, int lx, int ly, double gd,
                           double rho0, H16 h16) {
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
    Store<ST>::st(f, (size_t)q * plane + node, (CT)d, q, h16);
  }
}

// FP64 full populations <-> storage deviations.
template <class ST>
__global__ void k_pop_convert(void *fv, double *d64, size_t plane, int64_t nodes, double rho0,
                              int to_storage, H16 h16) {
  using CT = typename Store<ST>::CT;
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= nodes) return;
  ST *f = (ST *)fv;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double w = wq(q) * rho0;
    if (to_storage)
      Store<ST>::st(f, (size_t)q * plane + node, (CT)(d64[(size_t)q * nodes + node] - w), q, h16);
    else
      d64[(size_t)q * nodes + node] = w + (double)Store<ST>::ld(f, (size_t)q * plane + node, q, h16);
  }
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
      hipLaunchKernelGGL(k_init_pop<double>, grid, blk, 0, s->stream, s->f[b], s->plane, s->nodes, s->lx, s->ly, gd, s->rho0, s->h16);
    else if (s->precision == 1)
      hipLaunchKernelGGL(k_init_pop<float>, grid, blk, 0, s->stream, s->f[b], s->plane, s->nodes, s->lx, s->ly, gd, s->rho0, s->h16);
    else
      hipLaunchKernelGGL(k_init_pop<__half>, grid, blk, 0, s->stream, s->f[b], s->plane, s->nodes, s->lx, s->ly, gd, s->rho0, s->h16);
  }
  return hipGetLastError();
}

hipError_t launch_pop_convert(Sim *s, double *dev64, int to_storage) {
  dim3 grid((unsigned)((s->nodes + 255) / 256)), blk(256);
  void *f = s->f[s->cur];
  if (s->precision == 0)
    hipLaunchKernelGGL(k_pop_convert<double>, grid, blk, 0, s->stream, f, dev64, s->plane, s->nodes, s->rho0, to_storage, s->h16);
  else if (s->precision == 1)
    hipLaunchKernelGGL(k_pop_convert<float>, grid, blk, 0, s->stream, f, dev64, s->plane, s->nodes, s->rho0, to_storage, s->h16);
  else
    hipLaunchKernelGGL(k_pop_convert<__half>, grid, blk, 0, s->stream, f, dev64, s->plane, s->nodes, s->rho0, to_storage, s->h16);
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
  hipLaunchKernelGGL(k_link_enum, grid, blk, 0, s->stream, s->own, gown, s->nodes,
                     s->lx, s->ly, s->lz, out);
  return hipGetLastError();
}

}  // namespace susp
