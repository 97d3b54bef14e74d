// particles.hip -- sphere-side kernels for gfx950 (all geometry and forces in FP64).
//
//  k_cells_lds_ids cell list: cell of each sphere, counting sort, ascending ids per cell
//  k_pairs         Lees-Edwards cell search -> neighbour list (ascending ids, both
//                  directions), contact-at-start flags, spring history carried over (a wave
//                  per sphere; needs only the positions and the cell list)
//  k_pair_rev      each list entry's mirror entry; also the step's per-sphere link sums
//                  into F, T, S
//  k_substep       one DEM substep per sphere: contact (spring-dashpot + Cundall-Strack with
//                  Coulomb cap, Sec. 2), DLVO (eq. 13), lubrication (App. A), eq. (1)
//  k_map_update<1> new mapped-sphere footprints; fluid nodes covered by a sphere give it
//                  their mass and momentum
//  k_map_update<2> old footprints; released nodes are refilled at equilibrium with the
//                  surface velocity, the sphere pays that momentum; impulses applied
//  k_reduce        deterministic two-level stress reduction (eqs. 12, 14, 15) and the
//                  G', G'' quadratures (eqs. 17-18), its last work-group doing the second level
#include "susp_impl.h"

namespace susp {

__global__ void k_fill_i32(int32_t *p, size_t n, int32_t v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_f64(double *p, size_t n, double v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
hipError_t launch_fill_i32(int32_t *p, size_t n, int32_t v, hipStream_t st) {
  if (!n) return hipSuccess;
  size_t g = (n + 255) / 256;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_f64(double *p, size_t n, double v, hipStream_t st) {
  if (!n) return hipSuccess;
  size_t g = (n + 255) / 256;
  hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
__device__ inline int cell_of(const Cells &C, double x, double y, double z) {
  int a = (int)floor(x * C.ix), b = (int)floor(y * C.iy), c = (int)floor(z * C.iz);
  a = a < 0 ? 0 : (a >= C.nx ? C.nx - 1 : a);
  b = b < 0 ? 0 : (b >= C.ny ? C.ny - 1 : b);
  c = c < 0 ? 0 : (c >= C.nz ? C.nz - 1 : c);
  return a + C.nx * (b + C.ny * c);
}

// Arguments of the cell-list kernels (cnt: global counters of k_cells).
struct CellArgs {
  const double *R;
  int n;
  Cells C;
  int ncell;
  int32_t *start, *ids, *cnt;
};
#define SUSP_CELL_ARGS                                                                      \
  const double *R = A.R;                                                                    \
  const int n = A.n;                                                                        \
  const Cells C = A.C;                                                                      \
  const int ncell = A.ncell;                                                                \
  int32_t *start = A.start, *ids = A.ids;

// One work-group builds the whole cell list (counting sort, then ids sorted inside cells).
__device__ __forceinline__ void cells_wg(const CellArgs &A, int) {
  SUSP_CELL_ARGS
  int32_t *cnt = A.cnt;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int c = t; c < ncell; c += nt) cnt[c] = 0;
  __syncthreads();
  for (int i = t; i < n; i += nt) {
    const int c = cell_of(C, R[3 * i], R[3 * i + 1], R[3 * i + 2]);
    atomicAdd(&cnt[c], 1);
  }
  __syncthreads();
  // exclusive scan of cnt into start (chunked block scan)
  __shared__ int32_t part[1024];
  const int per = (ncell + nt - 1) / nt;
  const int c0 = t * per, c1 = min(ncell, c0 + per);
  int32_t sum = 0;
  for (int c = c0; c < c1; ++c) sum += cnt[c];
  part[t] = sum;
  __syncthreads();
  for (int o = 1; o < nt; o <<= 1) {
    int32_t v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int32_t run = t > 0 ? part[t - 1] : 0;
  for (int c = c0; c < c1; ++c) {
    const int32_t k = cnt[c];
    start[c] = run;
    cnt[c] = run;  // becomes the fill cursor
    run += k;
  }
  if (t == nt - 1) start[ncell] = part[nt - 1];
  __syncthreads();
  for (int i = t; i < n; i += nt) {
    const int c = cell_of(C, R[3 * i], R[3 * i + 1], R[3 * i + 2]);
    const int pos = atomicAdd(&cnt[c], 1);
    ids[pos] = i;
  }
  __syncthreads();
  for (int c = t; c < ncell; c += nt) {  // insertion sort inside each cell
    const int a = start[c], b = start[c + 1];
    for (int u = a + 1; u < b; ++u) {
      const int32_t v = ids[u];
      int w = u - 1;
      while (w >= a && ids[w] > v) { ids[w + 1] = ids[w]; --w; }
      ids[w + 1] = v;
    }
  }
}

// Same construction with the counters, the scan and the fill cursors in LDS (used when
// the cell grid fits: ncell <= LDS_CELLS).
constexpr int LDS_CELLS = 12288;
__device__ __forceinline__ void cells_lds_wg(const CellArgs &A, int) {
  SUSP_CELL_ARGS
  __shared__ int32_t cnt[LDS_CELLS];
  __shared__ int32_t part[1024];
  const int t = threadIdx.x, nt = blockDim.x;
  for (int c = t; c < ncell; c += nt) cnt[c] = 0;
  __syncthreads();
  for (int i = t; i < n; i += nt) atomicAdd(&cnt[cell_of(C, R[3 * i], R[3 * i + 1], R[3 * i + 2])], 1);
  __syncthreads();
  const int per = (ncell + nt - 1) / nt;
  const int c0 = t * per, c1 = min(ncell, c0 + per);
  int32_t sum = 0;
  for (int c = c0; c < c1; ++c) sum += cnt[c];
  part[t] = sum;
  __syncthreads();
  for (int o = 1; o < nt; o <<= 1) {
    int32_t v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int32_t run = t > 0 ? part[t - 1] : 0;
  for (int c = c0; c < c1; ++c) {
    const int32_t k = cnt[c];
    start[c] = run;
    cnt[c] = run;
    run += k;
  }
  if (t == nt - 1) start[ncell] = part[nt - 1];
  __syncthreads();
  for (int i = t; i < n; i += nt) {
    const int pos = atomicAdd(&cnt[cell_of(C, R[3 * i], R[3 * i + 1], R[3 * i + 2])], 1);
    ids[pos] = i;
  }
  __syncthreads();
  for (int c = t; c < ncell; c += nt) {  // insertion sort inside each cell
    const int a = start[c], b = start[c + 1];
    for (int u = a + 1; u < b; ++u) {
      const int32_t v = ids[u];
      int w = u - 1;
      while (w >= a && ids[w] > v) { ids[w + 1] = ids[w]; --w; }
      ids[w + 1] = v;
    }
  }
}

// The same list when the ids fit in LDS as well (n <= 16 x 1024): each thread keeps the cells
// of its (at most 16) spheres in registers, so positions are read once, and the fill and the
// sort inside each cell work in LDS; the ids are written out once at the end.
constexpr int LDS_IDS = 16 * 1024;
__device__ __forceinline__ void cells_lds_ids_wg(const CellArgs &A, int) {
  SUSP_CELL_ARGS
  __shared__ int32_t cnt[LDS_CELLS];
  __shared__ int32_t part[1024];
  __shared__ int32_t sid[LDS_IDS];
  const int t = threadIdx.x, nt = 1024;
  for (int c = t; c < ncell; c += nt) cnt[c] = 0;
  int cof[LDS_IDS / 1024];
#pragma unroll
  for (int k = 0; k < LDS_IDS / 1024; ++k) {
    const int i = t + k * nt;
    cof[k] = i < n ? cell_of(C, R[3 * i], R[3 * i + 1], R[3 * i + 2]) : 0;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < LDS_IDS / 1024; ++k)
    if (t + k * nt < n) atomicAdd(&cnt[cof[k]], 1);
  __syncthreads();
  const int per = (ncell + nt - 1) / nt;
  const int c0 = t * per, c1 = min(ncell, c0 + per);
  int32_t sum = 0;
  for (int c = c0; c < c1; ++c) sum += cnt[c];
  part[t] = sum;
  __syncthreads();
  for (int o = 1; o < nt; o <<= 1) {
    int32_t v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int32_t run = t > 0 ? part[t - 1] : 0;
  for (int c = c0; c < c1; ++c) {
    const int32_t k = cnt[c];
    start[c] = run;
    cnt[c] = run;
    run += k;
  }
  if (t == nt - 1) start[ncell] = part[nt - 1];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < LDS_IDS / 1024; ++k) {
    const int i = t + k * nt;
    if (i < n) sid[atomicAdd(&cnt[cof[k]], 1)] = i;
  }
  __syncthreads();
  // after the fill cnt[c] is the end of cell c, i.e. the start of cell c + 1
  for (int c = t; c < ncell; c += nt) {  // insertion sort inside each cell
    const int a = c > 0 ? cnt[c - 1] : 0, b = cnt[c];
    for (int u = a + 1; u < b; ++u) {
      const int32_t v = sid[u];
      int w = u - 1;
      while (w >= a && sid[w] > v) { sid[w + 1] = sid[w]; --w; }
      sid[w + 1] = v;
    }
  }
  __syncthreads();
  for (int i = t; i < n; i += nt) ids[i] = sid[i];
}

__global__ __launch_bounds__(1024) void k_cells(CellArgs A) { cells_wg(A, 0); }
__global__ __launch_bounds__(1024) void k_cells_m(const CellArgs *__restrict__ tab, const int32_t *__restrict__ pre,
                                                  int nj) {
  SUSP_MULTI_BODY(CellArgs, cells_wg);
}
__global__ __launch_bounds__(1024) void k_cells_lds(CellArgs A) { cells_lds_wg(A, 0); }
__global__ __launch_bounds__(1024) void k_cells_lds_m(const CellArgs *__restrict__ tab,
                                                      const int32_t *__restrict__ pre, int nj) {
  SUSP_MULTI_BODY(CellArgs, cells_lds_wg);
}
__global__ __launch_bounds__(1024) void k_cells_lds_ids(CellArgs A) { cells_lds_ids_wg(A, 0); }
__global__ __launch_bounds__(1024) void k_cells_lds_ids_m(const CellArgs *__restrict__ tab,
                                                          const int32_t *__restrict__ pre, int nj) {
  SUSP_MULTI_BODY(CellArgs, cells_lds_ids_wg);
}

hipError_t launch_cells(Sim *s, int32_t *cell_start, int32_t *cell_ids, int32_t *scratch) {
  CellArgs A;
  A.R = s->R[s->pcur];
  A.n = s->n;
  A.C = s->cells;
  A.ncell = s->ncell;
  A.start = cell_start;
  A.ids = cell_ids;
  A.cnt = scratch;
  // recorded for lockstep runs: the variant with its counters in global memory (4 KB of LDS),
  // which finds room beside other jobs' lattice work-groups; every variant builds the same
  // list (ids ascending within each cell)
  if (s->col) return dispatch(s, k_cells, k_cells_m, 1, 1024, A);
  if (s->ncell <= LDS_CELLS && s->n <= LDS_IDS) return dispatch(s, k_cells_lds_ids, k_cells_lds_ids_m, 1, 1024, A);
  if (s->ncell <= LDS_CELLS) return dispatch(s, k_cells_lds, k_cells_lds_m, 1, 1024, A);
  return dispatch(s, k_cells, k_cells_m, 1, 1024, A);
}

// Visit the distinct cells that can hold spheres within one cell width of (px,py,pz).
template <class F>
__device__ inline void near_cells(const Cells &C, const Box &b, double px, double py, double pz,
                                  F fn) {
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

// Pair geometry in the canonical order lo < hi: d = R_lo - R_hi (minimum image), k = image
// index of hi.  Both spheres of a pair evaluate exactly the same expression.
__device__ inline double pair_geo(const Box &b, const double *R, int lo, int hi, double &dx,
                                  double &dy, double &dz, int &k) {
  minimage(b, R[3 * lo] - R[3 * hi], R[3 * lo + 1] - R[3 * hi + 1], R[3 * lo + 2] - R[3 * hi + 2],
           dx, dy, dz, k);
  return dx * dx + dy * dy + dz * dz;
}

struct PairArgs {
  const double *R, *a, *amap;
  const int32_t *cell_start, *cell_ids;
  Cells C;
  Box b;             // static dimensions; offset from clk
  const Clock *clk;
  int n;
  double cutoff;
  int32_t *cnt, *nj;                 // new list
  const int32_t *ocnt, *onj;         // list of the previous step
  const double *oxi;                 // its final spring history
  const int32_t *oon;
  double *xi;                        // carried history for this step
  int32_t *on, *hstart;
  int32_t *flags;
};

// Neighbour list of one sphere per wave, four spheres per work-group.  The lanes take the
// candidates of the near cells in visiting order (cell by cell, each cell in its stored
// order); a ballot keeps those within the cutoff in that order (the first NCAP of them; more
// raise flag 4), and each kept partner goes to its rank among them, so the list ascends in
// partner id.  A pair that stays listed carries its spring history over from the previous
// list, where the lower id holds it.
__device__ __forceinline__ void pairs_wg(const PairArgs &A, const int bid) {
  __shared__ int32_t s_cs[4][32], s_pre[4][32], s_js[4][NCAP], s_srt[4][NCAP], s_old[4][NCAP];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = bid * 4 + wv;
  const bool ok = i < A.n;  // waves past the last sphere still reach the barriers
  const Box bx = clock_box(A.b, A.clk, 0);
  const double *R = A.R;
  // the near cells: lane k takes the k-th cell visited (at most 27)
  int ncv = 0, cell = -1;
  if (ok)
    near_cells(A.C, bx, R[3 * i], R[3 * i + 1], R[3 * i + 2], [&](int c) {
      if (ncv == lane) cell = c;
      ++ncv;
    });
  int cs = 0, cn = 0;
  if (cell >= 0) { cs = A.cell_start[cell]; cn = A.cell_start[cell + 1] - cs; }
  int incl = cn;  // inclusive scan of the cell counts over the lanes
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o, 64);
    if (lane >= o) incl += v;
  }
  const int total = __shfl(incl, 63, 64);
  if (lane < 32) { s_cs[wv][lane] = cs; s_pre[wv][lane] = incl - cn; }
  __syncthreads();
  int c = 0;
  bool ovl = false;
  for (int base = 0; base < total; base += 64) {
    const int t = base + lane;
    bool hit = false;
    int j = -1;
    if (t < total) {
      // the cell holding candidate t: the last one starting at or before t (a bisection over
      // the ncv <= 27 starts, which ascend)
      int k = 0;
#pragma unroll
      for (int step = 16; step > 0; step >>= 1)
        if (k + step < ncv && s_pre[wv][k + step] <= t) k += step;
      j = A.cell_ids[s_cs[wv][k] + (t - s_pre[wv][k])];
      if (j != i) {
        const int lo = i < j ? i : j, hi = i < j ? j : i;
        double dx, dy, dz;
        int kk;
        const double r2 = pair_geo(bx, R, lo, hi, dx, dy, dz, kk);
        const double rc = A.a[lo] + A.a[hi] + A.cutoff;
        hit = r2 < rc * rc;
        const double rm = A.amap[lo] + A.amap[hi];
        if (hit && r2 < rm * rm) ovl = true;
      }
    }
    const uint64_t m = __ballot(hit);
    const int pos = c + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    if (hit && pos < NCAP) s_js[wv][pos] = j;
    c += __popcll(m);
  }
  const int kept = c < NCAP ? c : NCAP;
  const int oc = ok ? A.ocnt[i] : 0;
  if (lane < oc) s_old[wv][lane] = A.onj[(size_t)i * NCAP + lane];
  __syncthreads();
  if (lane < kept) {  // rank among the kept partners (stable for equal ids)
    const int v = s_js[wv][lane];
    int r = 0;
    for (int w = 0; w < kept; ++w) {
      const int x = s_js[wv][w];
      r += (x < v || (x == v && w < lane)) ? 1 : 0;
    }
    s_srt[wv][r] = v;
  }
  __syncthreads();
  if (!ok) return;
  const uint64_t ov = __ballot(ovl);
  if (lane == 0) {
    if (c > NCAP) atomicOr(A.flags, 4);
    if (ov) atomicOr(A.flags, 1);
    A.cnt[i] = kept;
  }
  if (lane >= kept) return;
  const int j = s_srt[wv][lane];
  const size_t e = (size_t)i * NCAP + lane;
  A.nj[e] = j;
  if (j < i) return;  // the history of a pair lives with its lower id
  double x0 = 0, x1 = 0, x2 = 0;
  int on = 0;
  for (int v = 0; v < oc; ++v)
    if (s_old[wv][v] == j) {
      const size_t oe = (size_t)i * NCAP + v;
      if (A.oon[oe]) { x0 = A.oxi[3 * oe]; x1 = A.oxi[3 * oe + 1]; x2 = A.oxi[3 * oe + 2]; on = 1; }
      break;
    }
  A.xi[3 * e] = x0; A.xi[3 * e + 1] = x1; A.xi[3 * e + 2] = x2;
  A.on[e] = on;
  double dx, dy, dz;
  int k;
  const double r2 = pair_geo(bx, R, i, j, dx, dy, dz, k);
  A.hstart[e] = (sqrt(r2) - A.a[i] - A.a[j]) < 0.0 ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_pairs(PairArgs A) { pairs_wg(A, (int)blockIdx.x); }
__global__ __launch_bounds__(256) void k_pairs_m(const PairArgs *__restrict__ tab, const int32_t *__restrict__ pre,
                                                 int nj) {
  SUSP_MULTI_BODY(PairArgs, pairs_wg);
}

hipError_t launch_pairs(Sim *s, const Box &b) {
  PairArgs A;
  A.R = s->R[s->pcur]; A.a = s->a; A.amap = s->amap;
  A.cell_start = s->cell_start; A.cell_ids = s->cell_ids;
  A.C = s->cells; A.b = b; A.clk = s->clk; A.n = s->n; A.cutoff = s->pair_cutoff;
  const int nl = 1 - s->lcur;
  A.cnt = s->ncnt[nl]; A.nj = s->nj[nl];
  A.ocnt = s->ncnt[s->lcur]; A.onj = s->nj[s->lcur];
  A.oxi = s->hxi[s->hfin]; A.oon = s->hon[s->hfin];
  A.xi = s->hxi[1 - s->hfin]; A.on = s->hon[1 - s->hfin];
  A.hstart = s->hstart;
  A.flags = s->flags;
  if (s->n > 0) return dispatch(s, k_pairs, k_pairs_m, (s->n + 3) / 4, 256, A);
  return hipSuccess;
}

// ---------------------------------------------------------------------------------------
struct Phys {
  double kn, kt, eta_n, mu, delta, hc, F0, lambda, eta0, cutoff;
  int lub_sub;
};

// Squeeze coefficient zeta = eta0 X^A of the lubrication force on the sphere of radius ai
// (the X^A term of the pair expression below, App. A); 0 beyond h_c.
__device__ inline double lub_zeta(const Phys &P, double ai, double aj, double h) {
  if (!(h < P.hc)) return 0.0;
  const double PI = 3.14159265358979323846;
  const double hh = h > 0.0 ? h : 0.0;
  const double sa = ai + aj, s = 1.0 / sa;
  double inv = 0.5 * sa / (hh + P.delta);  // 1 / xi
  if (P.lub_sub) inv -= 0.5 * sa / (P.hc + P.delta);
  return P.eta0 * (12.0 * PI * (ai * ai) * (aj * aj) * (s * s * s) * inv);
}

__device__ inline void crs(double ax, double ay, double az, double bx, double by, double bz,
                           double &cx_, double &cy_, double &cz_) {
  cx_ = ay * bz - az * by;
  cy_ = az * bx - ax * bz;
  cz_ = ax * by - ay * bx;
}

// Scalar resistance functions of App. A for the block of a sphere of radius a against a partner
// of radius c (ratio b = c/a), at 1/xi (inv) and ln(1/xi) (lg).  With 1 + b = (a + c)/a the
// leading-order forms are polynomials in a, c and s = 1/(a + c), e.g. 6 pi a 2 b^2/(1 + b)^3 =
// 12 pi a^2 c^2 s^3: one division per pair for all of them.
struct LubF {
  double XA, YA, YB, XG, YG, YC, YCp, YH, YHp;
};
__device__ inline LubF lubf(double a, double c, double s, double inv, double lg) {
  const double PI = 3.14159265358979323846;
  const double a2 = a * a, c2 = c * c, s2 = s * s, s3 = s2 * s;
  LubF f;
  f.XA = 12.0 * PI * a2 * c2 * s3 * inv;
  f.YA = 1.6 * PI * a * c * (2.0 * a2 + a * c + 2.0 * c2) * s3 * lg;
  f.YB = 0.8 * PI * a2 * c * (4.0 * a + c) * s2 * lg;
  f.XG = 12.0 * PI * a2 * a * c2 * s3 * inv;
  f.YG = 0.4 * PI * a2 * c * (4.0 * a2 - a * c + 7.0 * c2) * s3 * lg;
  f.YC = 3.2 * PI * a2 * a * c * s * lg;
  f.YCp = 0.8 * PI * a2 * c2 * s * lg;
  f.YH = 0.8 * PI * a2 * a * c * (2.0 * a - c) * s2 * lg;
  f.YHp = 0.4 * PI * a2 * c2 * (a + 7.0 * c) * s2 * lg;
  return f;
}

// All pair forces of (lo, hi): force on lo F, torques Tl, Th, spring update, stresses.
struct PairOut {
  double F[3], Tl[3], Th[3];
  double vc[6], vr[6], sl[6];  // contact virial, DLVO virial (x -1/2 sym), stresslet sum
  double fnor, ft[3];          // contact: signed normal magnitude (+ apart), tangential force
  int on;
};

__device__ inline void sym_add(double *o, const double *a, const double *b, double w) {
  o[0] += w * (2.0 * a[0] * b[0]);
  o[1] += w * (2.0 * a[1] * b[1]);
  o[2] += w * (2.0 * a[2] * b[2]);
  o[3] += w * (a[0] * b[1] + b[0] * a[1]);
  o[4] += w * (a[0] * b[2] + b[0] * a[2]);
  o[5] += w * (a[1] * b[2] + b[1] * a[2]);
}

__device__ void pair_forces(const Phys &P, double ai, double aj, const double d[3],
                            const double *Ui, const double Uj[3], const double *Wi,
                            const double *Wj, double dt, double xi[3], int on_in, PairOut &o) {
  for (int c = 0; c < 3; ++c) { o.F[c] = 0; o.Tl[c] = 0; o.Th[c] = 0; o.ft[c] = 0; }
  for (int c = 0; c < 6; ++c) { o.vc[c] = 0; o.vr[c] = 0; o.sl[c] = 0; }
  o.fnor = 0;
  (void)on_in;
  const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  const double r = sqrt(r2);
  const double h = r - ai - aj;
  const double ir = 1.0 / r;
  const double n[3] = {d[0] * ir, d[1] * ir, d[2] * ir};
  const double Uij[3] = {Ui[0] - Uj[0], Ui[1] - Uj[1], Ui[2] - Uj[2]};
  double Fc[3] = {0, 0, 0};
  // ---- contact: normal spring-dashpot, tangential spring with Coulomb cap ----
  if (h < 0.0) {
    const double vn = -(Uij[0] * n[0] + Uij[1] * n[1] + Uij[2] * n[2]);
    const double fnm = P.kn * (-h) + P.eta_n * vn;
    const double Fn[3] = {fnm * n[0], fnm * n[1], fnm * n[2]};
    double awx = ai * Wi[0] + aj * Wj[0], awy = ai * Wi[1] + aj * Wj[1], awz = ai * Wi[2] + aj * Wj[2];
    double wnx, wny, wnz;
    crs(awx, awy, awz, n[0], n[1], n[2], wnx, wny, wnz);
    const double v[3] = {Uij[0] - wnx, Uij[1] - wny, Uij[2] - wnz};
    const double vdn = v[0] * n[0] + v[1] * n[1] + v[2] * n[2];
    const double vt[3] = {v[0] - vdn * n[0], v[1] - vdn * n[1], v[2] - vdn * n[2]};
    const double xn = xi[0] * n[0] + xi[1] * n[1] + xi[2] * n[2];
    const double xp[3] = {xi[0] - xn * n[0], xi[1] - xn * n[1], xi[2] - xn * n[2]};
    const double mo = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
    const double mp = sqrt(xp[0] * xp[0] + xp[1] * xp[1] + xp[2] * xp[2]);
    if (mp > 0.0) {
      const double sc = mo / mp;
      xi[0] = xp[0] * sc; xi[1] = xp[1] * sc; xi[2] = xp[2] * sc;
    } else {
      xi[0] = xp[0]; xi[1] = xp[1]; xi[2] = xp[2];
    }
    xi[0] += vt[0] * dt; xi[1] += vt[1] * dt; xi[2] += vt[2] * dt;
    double Ft[3] = {-P.kt * xi[0], -P.kt * xi[1], -P.kt * xi[2]};
    const double ftm = sqrt(Ft[0] * Ft[0] + Ft[1] * Ft[1] + Ft[2] * Ft[2]);
    const double cap = P.mu * fabs(fnm);
    if (ftm > cap) {
      const double sc = cap / ftm;
      Ft[0] *= sc; Ft[1] *= sc; Ft[2] *= sc;
      xi[0] = -Ft[0] / P.kt; xi[1] = -Ft[1] / P.kt; xi[2] = -Ft[2] / P.kt;
    }
    for (int c = 0; c < 3; ++c) Fc[c] = Fn[c] + Ft[c];
    crs(-ai * n[0], -ai * n[1], -ai * n[2], Ft[0], Ft[1], Ft[2], o.Tl[0], o.Tl[1], o.Tl[2]);
    crs(-aj * n[0], -aj * n[1], -aj * n[2], Ft[0], Ft[1], Ft[2], o.Th[0], o.Th[1], o.Th[2]);
    o.fnor = fnm;
    for (int c = 0; c < 3; ++c) o.ft[c] = Ft[c];
    o.on = 1;
  } else {
    xi[0] = xi[1] = xi[2] = 0.0;
    o.on = 0;
  }
  // ---- DLVO double-layer repulsion (eq. 13), gap clamped at contact ----
  double Fr[3] = {0, 0, 0};
  if (h < P.cutoff) {
    const double hh = h > 0.0 ? h : 0.0;
    const double f = P.F0 * exp(-hh / P.lambda);
    Fr[0] = f * n[0]; Fr[1] = f * n[1]; Fr[2] = f * n[2];
  }
  // ---- lubrication correction (App. A grand-resistance matrix, leading order) ----
  double Fl[3] = {0, 0, 0};
  if (h < P.hc) {
    const double hh = h > 0.0 ? h : 0.0;
    const double sa = ai + aj, s = 1.0 / sa;
    double inv = 0.5 * sa / (hh + P.delta);  // 1 / xi, xi = 2 (h + delta)/(ai + aj)
    double lg = log(inv);
    if (P.lub_sub) {  // minus the same at the cut-off h_c
      inv -= 0.5 * sa / (P.hc + P.delta);
      lg = log((P.hc + P.delta) / (hh + P.delta));
    }
    const LubF fi = lubf(ai, aj, s, inv, lg);
    const LubF fj = lubf(aj, ai, s, inv, lg);
    const double un = Uij[0] * n[0] + Uij[1] * n[1] + Uij[2] * n[2];
    double wix, wiy, wiz, wjx, wjy, wjz, ux_, uy_, uz_;
    crs(Wi[0], Wi[1], Wi[2], n[0], n[1], n[2], wix, wiy, wiz);
    crs(Wj[0], Wj[1], Wj[2], n[0], n[1], n[2], wjx, wjy, wjz);
    crs(Uij[0], Uij[1], Uij[2], n[0], n[1], n[2], ux_, uy_, uz_);
    const double Wixn[3] = {wix, wiy, wiz}, Wjxn[3] = {wjx, wjy, wjz}, Uxn[3] = {ux_, uy_, uz_};
    const double win = Wi[0] * n[0] + Wi[1] * n[1] + Wi[2] * n[2];
    const double wjn = Wj[0] * n[0] + Wj[1] * n[1] + Wj[2] * n[2];
    const double eta = P.eta0;
    for (int c = 0; c < 3; ++c) {
      const double AU = fi.XA * un * n[c] + fi.YA * (Uij[c] - un * n[c]);
      Fl[c] = -eta * (AU - fi.YB * Wixn[c] - fj.YB * Wjxn[c]);
      const double wip = Wi[c] - win * n[c], wjp = Wj[c] - wjn * n[c];
      o.Tl[c] += -eta * (fi.YB * Uxn[c] + fi.YC * wip + fi.YCp * wjp);
      o.Th[c] += -eta * (fj.YB * Uxn[c] + fi.YCp * wip + fj.YC * wjp);
    }
    double s1[6] = {0, 0, 0, 0, 0, 0}, s2[6] = {0, 0, 0, 0, 0, 0};
    double hi_[6] = {0, 0, 0, 0, 0, 0}, hj_[6] = {0, 0, 0, 0, 0, 0};
    sym_add(s1, n, n, 0.5 * un);
    s1[0] -= un / 3.0; s1[1] -= un / 3.0; s1[2] -= un / 3.0;
    sym_add(s2, n, Uij, 1.0);
    sym_add(s2, n, n, -un);
    sym_add(hi_, Wixn, n, 1.0);
    sym_add(hj_, Wjxn, n, 1.0);
    for (int c = 0; c < 6; ++c) {
      const double Si = -eta * (-(fi.XG * s1[c] + fi.YG * s2[c]) + fi.YH * hi_[c] + fi.YHp * hj_[c]);
      const double Sj = -eta * (-(fj.XG * s1[c] + fj.YG * s2[c]) + fj.YHp * hi_[c] + fj.YH * hj_[c]);
      o.sl[c] = Si + Sj;
    }
  }
  for (int c = 0; c < 3; ++c) o.F[c] = Fc[c] + Fr[c] + Fl[c];
  sym_add(o.vc, d, Fc, -0.5);
  sym_add(o.vr, d, Fr, -0.5);
}

// Entry of each neighbour-list slot that holds the pair's spring history (the slot of the
// lower id); one wave per sphere, lanes over its neighbour slots; the lower id's list
// ascends, so its slot is found by bisection.
struct RevArgs {
  const int32_t *cnt, *nj;
  int32_t *rev;
  unsigned long long *hacc;  // the step's fixed-point link sums [n][HYD][2] (cleared here)
  double *hyd;               // their values [n][HYD]
  int n;
};
__device__ __forceinline__ void pair_rev_wg(const RevArgs &A, const int bid) {
  const int32_t *cnt = A.cnt, *nj = A.nj;
  int32_t *rev = A.rev;
  const int n = A.n;
  const int i = bid * 4 + (threadIdx.x >> 6);
  const int u = threadIdx.x & 63;
  if (i < n && u < HYD) {  // the sphere's force, torque, stresslet and link count of the step
    const size_t k = (size_t)i * HYD + u;
    const long long h = (long long)A.hacc[2 * k], l = (long long)A.hacc[2 * k + 1];
    A.hyd[k] = ldexp((double)h, -FXH) + ldexp((double)l, -FXL);
    A.hacc[2 * k] = 0ull;
    A.hacc[2 * k + 1] = 0ull;
  }
  if (i >= n || u >= NCAP) return;
  if (u >= cnt[i]) return;
  const size_t e = (size_t)i * NCAP + u;
  const int j = nj[e];
  int r = (int)e;
  if (j < i) {
    const int32_t *lj = &nj[(size_t)j * NCAP];
    int lo = 0, hi = cnt[j];  // first slot holding an id >= i
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (lj[mid] < i) lo = mid + 1;
      else hi = mid;
    }
    r = lo < cnt[j] && lj[lo] == i ? j * NCAP + lo : -1;
  }
  rev[e] = r;
}

__global__ __launch_bounds__(256) void k_pair_rev(RevArgs A) { pair_rev_wg(A, (int)blockIdx.x); }
__global__ __launch_bounds__(256) void k_pair_rev_m(const RevArgs *__restrict__ tab, const int32_t *__restrict__ pre,
                                                    int nj) {
  SUSP_MULTI_BODY(RevArgs, pair_rev_wg);
}

hipError_t launch_pair_rev(Sim *s) {
  RevArgs A;
  A.cnt = s->ncnt[s->lcur];
  A.nj = s->nj[s->lcur];
  A.rev = s->rev;
  A.hacc = s->hacc;
  A.hyd = s->hyd[s->hcur];
  A.n = s->n;
  if (s->n > 0) return dispatch(s, k_pair_rev, k_pair_rev_m, (s->n + 3) / 4, 256, A);
  return hipSuccess;
}

struct SubArgs {
  const double *Ri, *Ui, *Wi, *Qi;
  double *Ro, *Uo, *Wo, *Qo;
  double *R0;
  const double *a, *m, *I;
  const double *hyd;
  const int32_t *cnt, *nj, *rev;
  const double *xin;
  const int32_t *onin;
  double *xout;
  int32_t *onout;
  double *pst;
  double *crec;     // contact records of the last substep (null: statistics off)
  int32_t *cflag;
  const int32_t *wmem;  // walls: membership (null: Lees-Edwards)
  double *wfs;          // walls: force on each wall sphere this step
  double *lb;           // implicit squeeze: right-hand side m U + dt (F^h + explicit forces)
  Phys P;
  Box b;             // static dimensions; offsets of this and the next step from clk
  const Clock *clk;
  double dts;
  int n, sub, last, quasi2d;
  int32_t *flags;
};

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// sum over the L lanes of a lane group (xor offsets stay inside the group)
template <int L> __device__ inline double gsum(double v) {
#pragma unroll
  for (int o = L / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double gsum16(double v) { return gsum<16>(v); }

// Contact statistics (Sec. 4.2, eqs. 19-23): record of a pair in contact at the last substep,
// kept in the lower id's entry: the in-plane unit direction n of d = R_lo - R_hi ((1, 0) if d
// has no in-plane part), F_nor and F_tan, the component along t = (-n_y, n_x) of the
// tangential force on the sphere at the tail of n (hi, which feels -ft): positive when it
// turns that sphere counterclockwise; it is the same seen from lo.  Flag 1 marks a record.
__device__ inline void record_contact(const SubArgs &A, size_t e, bool keep, const double d[3],
                                      const PairOut &o) {
  if (keep) {
    const double rxy = sqrt(d[0] * d[0] + d[1] * d[1]);
    double nx = 1.0, ny = 0.0;
    if (rxy > 0.0) { nx = d[0] / rxy; ny = d[1] / rxy; }
    A.crec[4 * e] = nx;
    A.crec[4 * e + 1] = ny;
    A.crec[4 * e + 2] = o.fnor;
    A.crec[4 * e + 3] = -(o.ft[0] * (-ny) + o.ft[1] * nx);
  }
  A.cflag[e] = keep ? 1 : 0;
}

// One DEM substep; SUB_L lanes per sphere, the lanes striding over the sphere's
// neighbours.  Both spheres of a pair evaluate the identical pair expression;
// the lower id owns the spring history and the pair's stress.
// REC: the last substep of a step with contact statistics on (records each contact).
// IMP: the normal squeeze part of each pair's lubrication force is left out here and taken
// at the new velocities by k_lub_sweep; this kernel then writes the right-hand side and the
// explicit first guess, and k_lub_advance moves the spheres.
constexpr int SUB_L = 4;  // lanes per sphere in k_substep
template <bool REC, bool IMP>
__device__ __forceinline__ void substep_wg(const SubArgs &A, const int bid) {
  const Box bx = clock_box(A.b, A.clk, 0);
  const double s1 = A.clk->cur.s1, ule1 = A.clk->cur.ule1;
  const int lane = threadIdx.x & 63;
  const int i = bid * (256 / SUB_L) + threadIdx.x / SUB_L;
  const int l = lane % SUB_L;
  const bool ok = i < A.n;
  double F[3] = {0, 0, 0}, T[3] = {0, 0, 0}, Fq[3] = {0, 0, 0}, st[PST];
#pragma unroll
  for (int c = 0; c < PST; ++c) st[c] = 0.0;
  const int c_i = ok ? A.cnt[i] : 0;
  for (int u = l; u < c_i; u += SUB_L) {
    const size_t own_e = (size_t)i * NCAP + u;
    const int j = A.nj[own_e];
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    const int re = A.rev[own_e];
    const size_t e = re >= 0 ? (size_t)re : own_e;
    double d[3];
    int k;
    pair_geo(bx, A.Ri, lo, hi, d[0], d[1], d[2], k);
    const double Uh[3] = {A.Ui[3 * hi] + k * bx.ule, A.Ui[3 * hi + 1], A.Ui[3 * hi + 2]};
    double xi[3] = {A.xin[3 * e], A.xin[3 * e + 1], A.xin[3 * e + 2]};
    PairOut o;
    pair_forces(A.P, A.a[lo], A.a[hi], d, &A.Ui[3 * lo], Uh, &A.Wi[3 * lo], &A.Wi[3 * hi], A.dts,
                xi, A.onin[e], o);
    double Fs[3] = {0.0, 0.0, 0.0};
    if (IMP) {  // the squeeze part -zeta n (n . (U_lo - U_hi)) of the lubrication force
      const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      const double nn[3] = {d[0] / r, d[1] / r, d[2] / r};
      const double z = lub_zeta(A.P, A.a[lo], A.a[hi], r - A.a[lo] - A.a[hi]);
      const double un = nn[0] * (A.Ui[3 * lo] - Uh[0]) + nn[1] * (A.Ui[3 * lo + 1] - Uh[1]) +
                        nn[2] * (A.Ui[3 * lo + 2] - Uh[2]);
      for (int c = 0; c < 3; ++c) Fs[c] = -z * un * nn[c];
    }
    if (i == lo) {
      for (int c = 0; c < 3; ++c) { F[c] += o.F[c] - Fs[c]; T[c] += o.Tl[c]; Fq[c] += Fs[c]; }
      A.xout[3 * e] = xi[0]; A.xout[3 * e + 1] = xi[1]; A.xout[3 * e + 2] = xi[2];
      A.onout[e] = o.on;
      for (int c = 0; c < 6; ++c) { st[c] += o.sl[c]; st[6 + c] += o.vc[c]; st[12 + c] += o.vr[c]; }
    } else {
      for (int c = 0; c < 3; ++c) { F[c] -= o.F[c] - Fs[c]; T[c] += o.Th[c]; Fq[c] -= Fs[c]; }
    }
    if (REC) record_contact(A, own_e, i == lo && o.on, d, o);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) { F[c] = gsum<SUB_L>(F[c]); T[c] = gsum<SUB_L>(T[c]); }
  if (IMP) {
#pragma unroll
    for (int c = 0; c < 3; ++c) Fq[c] = gsum<SUB_L>(Fq[c]);
  }
#pragma unroll
  for (int c = 0; c < PST; ++c) st[c] = gsum<SUB_L>(st[c]);
  if (!ok || l != 0) return;
  if (A.sub == 0) {
    for (int c = 0; c < 3; ++c) A.R0[3 * i + c] = A.Ri[3 * i + c];
  } else {
    for (int c = 0; c < PST; ++c) st[c] += A.pst[(size_t)i * PST + c];
  }
  for (int c = 0; c < PST; ++c) A.pst[(size_t)i * PST + c] = st[c];
  if (A.wmem && A.wmem[i] > 0) {
    // a wall sphere moves with its wall (Sec. 3); its hydrodynamic force and the
    // substep mean of its pair forces load the wall
    const double sg = A.wmem[i] == 2 ? 1.0 : -1.0;
    for (int c = 0; c < 3; ++c) {
      const double f = F[c] * A.dts;
      A.wfs[3 * i + c] = A.sub == 0 ? A.hyd[(size_t)i * HYD + c] + f : A.wfs[3 * i + c] + f;
    }
    const double u = sg * (A.last ? A.clk->cur.uw1 : A.clk->cur.uw);
    A.Ro[3 * i] = A.Ri[3 * i] + A.dts * (sg * A.clk->cur.uw);
    A.Ro[3 * i + 1] = A.Ri[3 * i + 1];
    A.Ro[3 * i + 2] = A.Ri[3 * i + 2];
    if (A.last) {
      for (int it = 0; it < 4 && A.Ro[3 * i] >= bx.Lx; ++it) A.Ro[3 * i] -= bx.Lx;
      for (int it = 0; it < 4 && A.Ro[3 * i] < 0.0; ++it) A.Ro[3 * i] += bx.Lx;
    }
    A.Uo[3 * i] = u; A.Uo[3 * i + 1] = 0.0; A.Uo[3 * i + 2] = 0.0;
    A.Wo[3 * i] = 0.0; A.Wo[3 * i + 1] = 0.0; A.Wo[3 * i + 2] = 0.0;
    for (int c = 0; c < 4; ++c) A.Qo[4 * i + c] = A.Qi[4 * i + c];
    return;
  }
  if (IMP) {
    // spin and orientation as usual; the velocity's right-hand side and explicit first
    // guess for the sweeps; the position waits for the solved velocity (k_lub_advance)
    double W[3];
    for (int c = 0; c < 3; ++c) {
      const double fh = A.hyd[(size_t)i * HYD + c];
      A.lb[3 * i + c] = A.m[i] * A.Ui[3 * i + c] + A.dts * (fh + F[c]);
      A.Uo[3 * i + c] = A.Ui[3 * i + c] + A.dts * (fh + F[c] + Fq[c]) / A.m[i];
      W[c] = A.Wi[3 * i + c] + A.dts * (A.hyd[(size_t)i * HYD + 3 + c] + T[c]) / A.I[i];
      A.Ro[3 * i + c] = A.Ri[3 * i + c];
    }
    if (A.quasi2d) { W[0] = 0.0; W[1] = 0.0; }
    double qw = A.Qi[4 * i], qx = A.Qi[4 * i + 1], qy = A.Qi[4 * i + 2], qz = A.Qi[4 * i + 3];
    const double dw = -(W[0] * qx + W[1] * qy + W[2] * qz);
    const double dx = W[0] * qw + (W[1] * qz - W[2] * qy);
    const double dy = W[1] * qw + (W[2] * qx - W[0] * qz);
    const double dz = W[2] * qw + (W[0] * qy - W[1] * qx);
    qw += 0.5 * A.dts * dw; qx += 0.5 * A.dts * dx; qy += 0.5 * A.dts * dy; qz += 0.5 * A.dts * dz;
    const double nn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    for (int c = 0; c < 3; ++c) A.Wo[3 * i + c] = W[c];
    A.Qo[4 * i] = qw / nn; A.Qo[4 * i + 1] = qx / nn; A.Qo[4 * i + 2] = qy / nn; A.Qo[4 * i + 3] = qz / nn;
    return;
  }
  // eq. (1), symplectic Euler with the hydrodynamic force and torque of this step
  double U[3], W[3], R[3];
  for (int c = 0; c < 3; ++c) {
    U[c] = A.Ui[3 * i + c] + A.dts * (A.hyd[(size_t)i * HYD + c] + F[c]) / A.m[i];
    W[c] = A.Wi[3 * i + c] + A.dts * (A.hyd[(size_t)i * HYD + 3 + c] + T[c]) / A.I[i];
  }
  if (A.quasi2d) { U[2] = 0.0; W[0] = 0.0; W[1] = 0.0; }
  for (int c = 0; c < 3; ++c) R[c] = A.Ri[3 * i + c] + A.dts * U[c];
  // orientation: q <- normalize(q + dt/2 (0, W) (x) q)
  double qw = A.Qi[4 * i], qx = A.Qi[4 * i + 1], qy = A.Qi[4 * i + 2], qz = A.Qi[4 * i + 3];
  const double dw = -(W[0] * qx + W[1] * qy + W[2] * qz);
  const double dx = W[0] * qw + (W[1] * qz - W[2] * qy);
  const double dy = W[1] * qw + (W[2] * qx - W[0] * qz);
  const double dz = W[2] * qw + (W[0] * qy - W[1] * qx);
  qw += 0.5 * A.dts * dw; qx += 0.5 * A.dts * dx; qy += 0.5 * A.dts * dy; qz += 0.5 * A.dts * dz;
  const double nn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  if (A.last) {  // Lees-Edwards wrap with the offset of the next step (none with walls)
    if (A.wmem) {
    } else if (R[1] >= bx.Ly) { R[1] -= bx.Ly; R[0] -= s1; U[0] -= ule1; }
    else if (R[1] < 0.0) { R[1] += bx.Ly; R[0] += s1; U[0] += ule1; }
    for (int it = 0; it < 4 && R[0] >= bx.Lx; ++it) R[0] -= bx.Lx;
    for (int it = 0; it < 4 && R[0] < 0.0; ++it) R[0] += bx.Lx;
    for (int it = 0; it < 4 && R[2] >= bx.Lz; ++it) R[2] -= bx.Lz;
    for (int it = 0; it < 4 && R[2] < 0.0; ++it) R[2] += bx.Lz;
  }
  for (int c = 0; c < 3; ++c) { A.Uo[3 * i + c] = U[c]; A.Wo[3 * i + c] = W[c]; A.Ro[3 * i + c] = R[c]; }
  A.Qo[4 * i] = qw / nn; A.Qo[4 * i + 1] = qx / nn; A.Qo[4 * i + 2] = qy / nn; A.Qo[4 * i + 3] = qz / nn;
  if (A.last) {  // non-finite, or a runaway the bounded wraps could not bring back
    bool ok = true;
    for (int c = 0; c < 3; ++c) ok = ok && isfinite(R[c]) && isfinite(U[c]) && isfinite(W[c]);
    ok = ok && R[0] > -bx.Lx && R[0] < 2.0 * bx.Lx && R[1] > -bx.Ly && R[1] < 2.0 * bx.Ly &&
         R[2] > -bx.Lz && R[2] < 2.0 * bx.Lz;
    if (A.wmem) ok = ok && R[1] >= 0.0 && R[1] < bx.Ly;  // walls: a sphere left the gap
    if (!ok) atomicOr(A.flags, 2);
  }
}

// One Jacobi sweep of the implicit squeeze terms: for every free sphere
// (m I + dt sum zeta n n) U_i = b_i + dt sum zeta n (n . U_partner) with the partners'
// velocities from the previous sweep (16 lanes per sphere over its neighbours, shuffle sums
// in a fixed order, a 3x3 solve by Cramer's rule); wall spheres keep theirs.
struct SweepArgs {
  const double *Ri, *a, *m, *lb;
  const int32_t *cnt, *nj, *wmem;
  const double *Uin;
  double *Uout;
  Phys P;
  Box b;
  const Clock *clk;
  double dts;
  int n;
};

__global__ __launch_bounds__(256) void k_lub_sweep(SweepArgs A) {
  const Box bx = clock_box(A.b, A.clk, 0);
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 16 + (threadIdx.x >> 4);
  const int l = lane & 15;
  const bool ok = i < A.n;
  double M[6] = {0, 0, 0, 0, 0, 0}, r[3] = {0, 0, 0};  // xx yy zz xy xz yz
  const int c_i = ok ? A.cnt[i] : 0;
  for (int u = l; u < c_i; u += 16) {
    const int j = A.nj[(size_t)i * NCAP + u];
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    double d[3];
    int k;
    pair_geo(bx, A.Ri, lo, hi, d[0], d[1], d[2], k);
    const double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double z = lub_zeta(A.P, A.a[lo], A.a[hi], rr - A.a[lo] - A.a[hi]);
    if (z == 0.0) continue;
    const double n[3] = {d[0] / rr, d[1] / rr, d[2] / rr};
    // the partner's image: hi's moves at U_hi + k U_LE, lo's (seen from hi) at U_lo - k U_LE
    const double sx = i == lo ? k * bx.ule : -k * bx.ule;
    const double up = n[0] * (A.Uin[3 * j] + sx) + n[1] * A.Uin[3 * j + 1] + n[2] * A.Uin[3 * j + 2];
    const double w = A.dts * z;
    M[0] += w * n[0] * n[0]; M[1] += w * n[1] * n[1]; M[2] += w * n[2] * n[2];
    M[3] += w * n[0] * n[1]; M[4] += w * n[0] * n[2]; M[5] += w * n[1] * n[2];
    for (int c = 0; c < 3; ++c) r[c] += w * n[c] * up;
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) M[c] = gsum16(M[c]);
#pragma unroll
  for (int c = 0; c < 3; ++c) r[c] = gsum16(r[c]);
  if (!ok || l != 0) return;
  if (A.wmem && A.wmem[i] > 0) {
    for (int c = 0; c < 3; ++c) A.Uout[3 * i + c] = A.Uin[3 * i + c];
    return;
  }
  const double mi = A.m[i];
  const double a00 = mi + M[0], a11 = mi + M[1], a22 = mi + M[2], a01 = M[3], a02 = M[4], a12 = M[5];
  const double b0 = A.lb[3 * i] + r[0], b1 = A.lb[3 * i + 1] + r[1], b2 = A.lb[3 * i + 2] + r[2];
  const double c00 = a11 * a22 - a12 * a12, c01 = a12 * a02 - a01 * a22, c02 = a01 * a12 - a11 * a02;
  const double det = a00 * c00 + a01 * c01 + a02 * c02;
  const double c11 = a00 * a22 - a02 * a02, c12 = a02 * a01 - a00 * a12, c22 = a00 * a11 - a01 * a01;
  A.Uout[3 * i] = (c00 * b0 + c01 * b1 + c02 * b2) / det;
  A.Uout[3 * i + 1] = (c01 * b0 + c11 * b1 + c12 * b2) / det;
  A.Uout[3 * i + 2] = (c02 * b0 + c12 * b1 + c22 * b2) / det;
}

// The solved velocity moves the sphere (and, on a step's last substep, the Lees-Edwards and
// periodic wraps and the checks of k_substep); wall spheres moved in k_substep.
__global__ __launch_bounds__(256) void k_lub_advance(SubArgs A, const double *Ufin) {
  const Box bx = clock_box(A.b, A.clk, 0);
  const double s1 = A.clk->cur.s1, ule1 = A.clk->cur.ule1;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  if (A.wmem && A.wmem[i] > 0) return;
  double U[3], R[3];
  for (int c = 0; c < 3; ++c) U[c] = Ufin[3 * i + c];
  if (A.quasi2d) U[2] = 0.0;
  for (int c = 0; c < 3; ++c) R[c] = A.Ri[3 * i + c] + A.dts * U[c];
  if (A.last) {
    if (A.wmem) {
    } else if (R[1] >= bx.Ly) { R[1] -= bx.Ly; R[0] -= s1; U[0] -= ule1; }
    else if (R[1] < 0.0) { R[1] += bx.Ly; R[0] += s1; U[0] += ule1; }
    for (int it = 0; it < 4 && R[0] >= bx.Lx; ++it) R[0] -= bx.Lx;
    for (int it = 0; it < 4 && R[0] < 0.0; ++it) R[0] += bx.Lx;
    for (int it = 0; it < 4 && R[2] >= bx.Lz; ++it) R[2] -= bx.Lz;
    for (int it = 0; it < 4 && R[2] < 0.0; ++it) R[2] += bx.Lz;
  }
  for (int c = 0; c < 3; ++c) { A.Uo[3 * i + c] = U[c]; A.Ro[3 * i + c] = R[c]; }
  if (A.last) {
    bool ok = true;
    for (int c = 0; c < 3; ++c) ok = ok && isfinite(R[c]) && isfinite(U[c]) && isfinite(A.Wo[3 * i + c]);
    ok = ok && R[0] > -bx.Lx && R[0] < 2.0 * bx.Lx && R[1] > -bx.Ly && R[1] < 2.0 * bx.Ly &&
         R[2] > -bx.Lz && R[2] < 2.0 * bx.Lz;
    if (A.wmem) ok = ok && R[1] >= 0.0 && R[1] < bx.Ly;
    if (!ok) atomicOr(A.flags, 2);
  }
}
template <bool REC, bool IMP>
__global__ __launch_bounds__(256, 2) void k_substep(SubArgs A) { substep_wg<REC, IMP>(A, (int)blockIdx.x); }
template <bool REC, bool IMP>
__global__ __launch_bounds__(256, 2) void k_substep_m(const SubArgs *__restrict__ tab, const int32_t *__restrict__ pre,
                                                      int nj) {
  SUSP_MULTI_BODY(SubArgs, (substep_wg<REC, IMP>));
}

hipError_t launch_substep(Sim *s, const Box &b, int sub) {
  SubArgs A;
  const int pi = s->pcur, po = 1 - s->pcur;
  A.Ri = s->R[pi]; A.Ui = s->U[pi]; A.Wi = s->W[pi]; A.Qi = s->Q[pi];
  A.Ro = s->R[po]; A.Uo = s->U[po]; A.Wo = s->W[po]; A.Qo = s->Q[po];
  A.R0 = s->R0;
  A.a = s->a; A.m = s->m; A.I = s->I;
  A.hyd = s->hyd[s->hcur];
  A.cnt = s->ncnt[s->lcur]; A.nj = s->nj[s->lcur]; A.rev = s->rev;
  // history ping-pong: substep k reads buffer (start + k) % 2
  const int hin = (1 - s->hfin + sub) & 1;
  A.xin = s->hxi[hin]; A.onin = s->hon[hin];
  A.xout = s->hxi[1 - hin]; A.onout = s->hon[1 - hin];
  A.pst = s->pst;
  A.crec = s->cbins > 0 ? s->crec : nullptr;
  A.wmem = s->boundary == 1 ? s->wmem : nullptr;
  A.wfs = s->wfs;
  A.cflag = s->cflag;
  A.P.kn = s->kn; A.P.kt = s->kt; A.P.eta_n = s->eta_n; A.P.mu = s->mu;
  A.P.delta = s->lub_delta; A.P.hc = s->lub_hc; A.P.F0 = s->F0; A.P.lambda = s->lambda;
  A.P.eta0 = s->eta0; A.P.cutoff = s->pair_cutoff; A.P.lub_sub = s->lub_sub;
  A.b = b;
  A.dts = 1.0 / (double)s->n_sub;
  A.clk = s->clk;
  A.n = s->n; A.sub = sub; A.last = sub == s->n_sub - 1; A.quasi2d = s->quasi2d;
  A.flags = s->flags;
  A.lb = s->lb;
  if (s->n > 0) {
    const int per = 256 / SUB_L;
    const dim3 gs((s->n + per - 1) / per), g((s->n + 15) / 16), blk(256);
    const bool rec = A.crec && A.last;
    if (s->lub_implicit == 0) {
      if (rec) return dispatch(s, k_substep<true, false>, k_substep_m<true, false>, gs.x, 256, A);
      return dispatch(s, k_substep<false, false>, k_substep_m<false, false>, gs.x, 256, A);
    } else {
      SUSP_NO_COLLECT(s);
      if (rec) hipLaunchKernelGGL((k_substep<true, true>), gs, blk, 0, s->stream, A);
      else hipLaunchKernelGGL((k_substep<false, true>), gs, blk, 0, s->stream, A);
      // Jacobi sweeps between the new velocity buffer and the scratch buffer
      SweepArgs W;
      W.Ri = A.Ri; W.a = A.a; W.m = A.m; W.lb = s->lb;
      W.cnt = A.cnt; W.nj = A.nj; W.wmem = A.wmem;
      W.P = A.P; W.b = A.b; W.clk = A.clk; W.dts = A.dts; W.n = s->n;
      double *buf[2] = {A.Uo, s->uimp};
      for (int k = 0; k < s->lub_implicit; ++k) {
        W.Uin = buf[k & 1];
        W.Uout = buf[(k + 1) & 1];
        hipLaunchKernelGGL(k_lub_sweep, g, blk, 0, s->stream, W);
      }
      hipLaunchKernelGGL(k_lub_advance, dim3((s->n + 255) / 256), dim3(256), 0, s->stream, A,
                         (const double *)buf[s->lub_implicit & 1]);
    }
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Candidate boxes of a sphere's mapped footprint: three Lees-Edwards image boxes.
struct Foot {
  int xlo[3], nxk[3], ylo[3], nyk[3], zlo, nzk;
  int tot[3];
};

__device__ inline void cand(double c, double r, int L, int &lo, int &cnt) {
  int a = (int)ceil(c - r - 1e-6), b = (int)floor(c + r + 1e-6);
  if (b - a + 1 >= L) { a = 0; b = L - 1; }
  lo = a;
  cnt = b - a + 1;
}

__device__ inline void footprint(const Box &bx, const double *R, int p, double r, Foot &f) {
  cand(R[3 * p + 2], r, bx.lz, f.zlo, f.nzk);
  for (int k = -1; k <= 1; ++k) {
    const double cyy = R[3 * p + 1] + k * bx.Ly;
    const double cxx = R[3 * p] + k * bx.s;
    int ylo = (int)ceil(cyy - r - 1e-6), yhi = (int)floor(cyy + r + 1e-6);
    if (ylo < 0) ylo = 0;
    if (yhi > bx.ly - 1) yhi = bx.ly - 1;
    const int t = k + 1;
    f.ylo[t] = ylo;
    f.nyk[t] = yhi >= ylo ? yhi - ylo + 1 : 0;
    cand(cxx, r, bx.lx, f.xlo[t], f.nxk[t]);
    f.tot[t] = f.nyk[t] * f.nxk[t] * f.nzk;
  }
}

// Decode candidate t; returns true with the node and its displacement if inside sphere p.
__device__ inline bool foot_node(const Box &bx, const double *R, int p, double r, const Foot &f,
                                 int t, int64_t &node, double d[3], int &kk) {
  int k = 0;
  while (t >= f.tot[k]) { t -= f.tot[k]; ++k; }
  const int nx = f.nxk[k], ny = f.nyk[k];
  const int ix = t % nx;
  const int iy = (t / nx) % ny;
  const int iz = t / (nx * ny);
  int x = f.xlo[k] + ix, y = f.ylo[k] + iy, z = f.zlo + iz;
  x %= bx.lx; x = x < 0 ? x + bx.lx : x;
  z %= bx.lz; z = z < 0 ? z + bx.lz : z;
  minimage(bx, (double)x - R[3 * p], (double)y - R[3 * p + 1], (double)z - R[3 * p + 2], d[0],
           d[1], d[2], kk);
  if (kk != k - 1) return false;
  if (!(d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < r * r)) return false;
  node = x + (int64_t)bx.lx * (y + (int64_t)bx.ly * z);
  return true;
}

// Full mapping of every sphere into an all-fluid map (creation and state loads).
struct MapFullArgs {
  const double *R, *amap;
  int32_t *own;
  Box b;
  int32_t *flags;
};

__global__ __launch_bounds__(256) void k_map_full(MapFullArgs A) {
  const int p = blockIdx.x;
  const double r = A.amap[p];
  if (!(isfinite(A.R[3 * p]) && isfinite(A.R[3 * p + 1]) && isfinite(A.R[3 * p + 2]))) {
    if (threadIdx.x == 0) atomicOr(A.flags, 2);
    return;
  }
  Foot f;
  footprint(A.b, A.R, p, r, f);
  const int tot = f.tot[0] + f.tot[1] + f.tot[2];
  for (int t = threadIdx.x; t < tot; t += blockDim.x) {
    int64_t node;
    double d[3];
    int kk;
    if (!foot_node(A.b, A.R, p, r, f, t, node, d, kk)) continue;
    const int32_t old = atomicCAS(&A.own[node], -1, p);
    if (old != -1 && old != p) { atomicMin(&A.own[node], p); atomicOr(A.flags, 1); }
  }
}

hipError_t launch_map_full(Sim *s, const Box &b) {
  MapFullArgs A;
  A.R = s->R[s->pcur]; A.amap = s->amap; A.own = s->own; A.b = b; A.flags = s->flags;
  if (s->n > 0) hipLaunchKernelGGL(k_map_full, dim3(s->n), dim3(256), 0, s->stream, A);
  return hipGetLastError();
}

// In-place map update after the spheres moved.  A node can change owner only if its
// distance d from (an image of) a sphere lies within delta of the mapped radius, delta
// = the sphere's displacement plus the change of the Lees-Edwards offset; each sphere
// visits that shell row by row (two short x-intervals per row) through its new images.
// Phase 1 claims nodes that entered the sphere: a fluid node is covered (its fluid mass
// and momentum go to the sphere); a node handed over by a sphere that left it changes
// owner without a fluid event.  Phase 2 releases nodes that left the sphere and were not
// claimed: they are refilled with the equilibrium at rho0 and the surface velocity, which
// the sphere pays; then the impulses of both phases are applied.
struct MapArgs {
  const double *R, *U, *W;  // state after the move
  const double *R0;         // positions before the move
  const double *amap, *m, *I;
  double *Uw, *Ww;
  int32_t *own;
  void *f;
  size_t plane;
  Box b;             // static dimensions; offsets before and after the step from clk
  const Clock *clk;
  double rho0;
  int quasi2d;
  double *dp;
  int32_t *flags;
  H16 h16;
  const int32_t *wmem;  // walls: membership (null: Lees-Edwards)
};

__device__ inline bool inside_new(const MapArgs &A, const Box &bnew, int v, double x, double y, double z) {
  double d0, d1, d2;
  int k;
  minimage(bnew, x - A.R[3 * v], y - A.R[3 * v + 1], z - A.R[3 * v + 2], d0, d1, d2, k);
  return d0 * d0 + d1 * d1 + d2 * d2 < A.amap[v] * A.amap[v];
}

template <class ST, int PHASE>
__device__ __forceinline__ void map_update_wg(const MapArgs &A, const int bid) {
  using CT = typename Store<ST>::CT;
  const Box bnew = clock_box(A.b, A.clk, 1), bold = clock_box(A.b, A.clk, 0);
  const int p = bid;
  const int lane = threadIdx.x;
  const double *Rn = &A.R[3 * p], *Ro = &A.R0[3 * p];
  if (!(isfinite(Rn[0]) && isfinite(Rn[1]) && isfinite(Rn[2]) && isfinite(Ro[0]) &&
        isfinite(Ro[1]) && isfinite(Ro[2]))) {
    if (lane == 0) atomicOr(A.flags, 2);
    return;
  }
  const double a = A.amap[p];
  const double a2 = a * a;
  double e0, e1, e2;
  int ke;
  minimage(bnew, Rn[0] - Ro[0], Rn[1] - Ro[1], Rn[2] - Ro[2], e0, e1, e2, ke);
  const double disp = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
  if (!(disp <= 1.0)) {  // a blown-up run: more than a node per step (the shell would be huge)
    if (lane == 0) atomicOr(A.flags, 16);
    return;
  }
  // change of the Lees-Edwards offset, taken modulo the period (the offset wraps at Lx)
  double ds = bnew.s - bold.s;
  ds -= bnew.Lx * rint(ds / bnew.Lx);
  // a node changes owner only within delta of the surface: the displacement, plus the offset
  // change for the images across the sliding plane (all images when the sphere itself crossed
  // it this step)
  const bool crossed = fabs(Rn[1] - Ro[1]) > 0.5 * bnew.Ly;
  const double delta1 = disp + fabs(ds) + 1e-6;
  const double delta0 = crossed ? delta1 : disp + 1e-6;
  const double ro = a + delta1;  // the widest shell, for the row bounds in z
  const Box &B = bnew;
  // rows (y, z) of the shell around each image of the new position
  int zlo = (int)floor(Rn[2] - ro), zhi = (int)ceil(Rn[2] + ro);
  const bool zall = zhi - zlo + 1 >= B.lz;
  if (zall) { zlo = 0; zhi = B.lz - 1; }
  const int nz = zhi - zlo + 1;
  int ylo[3], ny[3];
  int rows = 0;
  for (int k = -1; k <= 1; ++k) {
    const double cyy = Rn[1] + k * B.Ly;
    const double rok = a + (k == 0 ? delta0 : delta1);
    int lo = (int)floor(cyy - rok), hi = (int)ceil(cyy + rok);
    if (lo < 0) lo = 0;
    if (hi > B.ly - 1) hi = B.ly - 1;
    ylo[k + 1] = lo;
    ny[k + 1] = hi >= lo ? hi - lo + 1 : 0;
    rows += ny[k + 1] * nz;
  }
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  // row r: image kb (rows of image 0 first), then t = z index * ny + y index within it; the
  // quotient by ny through a float reciprocal (exact: t < 2^16 keeps (t + 1/2) / ny at least
  // 1/(2 ny) away from an integer, far beyond the float error)
  const int n0 = ny[0] * nz, n01 = n0 + ny[1] * nz;
  const float inv0 = 1.0f / (float)max(ny[0], 1), inv1 = 1.0f / (float)max(ny[1], 1),
              inv2 = 1.0f / (float)max(ny[2], 1);
  for (int r = lane; r < rows; r += 64) {
    const int kb = r < n0 ? 0 : (r < n01 ? 1 : 2);
    const int t = r - (kb == 0 ? 0 : (kb == 1 ? n0 : n01));
    const int nyk = kb == 0 ? ny[0] : (kb == 1 ? ny[1] : ny[2]);
    const float invk = kb == 0 ? inv0 : (kb == 1 ? inv1 : inv2);
    const int zi = (int)(((float)t + 0.5f) * invk);
    const int k = kb - 1;
    const int y = (kb == 0 ? ylo[0] : (kb == 1 ? ylo[1] : ylo[2])) + (t - zi * nyk);
    const int zu = zlo + zi;
    int z = zu % B.lz;
    z = z < 0 ? z + B.lz : z;
    const double cxx = Rn[0] + k * B.s;
    const double dk = k == 0 ? delta0 : delta1;
    const double ro = a + dk, ri = a - dk;
    const double dyy = (double)y - (Rn[1] + k * B.Ly);
    const double dzz = zall ? 0.0 : (double)zu - Rn[2];
    const double oo = ro * ro - dyy * dyy - dzz * dzz;
    if (!zall && oo < 0.0) continue;
    // candidate x-intervals of this row (all x when the row is not bounded)
    int xa0, xa1, xb0 = 1, xb1 = 0;
    if (zall) {
      xa0 = (int)ceil(cxx - ro - 1e-6); xa1 = (int)floor(cxx + ro + 1e-6);
    } else {
      const double xo = sqrt(oo);
      const double ii = ri > 0.0 ? ri * ri - dyy * dyy - dzz * dzz : -1.0;
      if (ii <= 0.0) {
        xa0 = (int)ceil(cxx - xo - 1e-6); xa1 = (int)floor(cxx + xo + 1e-6);
      } else {
        const double xi = sqrt(ii);
        xa0 = (int)ceil(cxx - xo - 1e-6); xa1 = (int)floor(cxx - xi + 1e-6);
        xb0 = (int)ceil(cxx + xi - 1e-6); xb1 = (int)floor(cxx + xo + 1e-6);
      }
    }
    if (xa1 - xa0 + 1 >= B.lx || (xb1 >= xb0 && xb1 - xa0 + 1 >= B.lx)) {
      xa0 = 0; xa1 = B.lx - 1; xb0 = 1; xb1 = 0;  // whole row, once
    }
    for (int seg = 0; seg < 2; ++seg) {
      const int x0 = seg == 0 ? xa0 : xb0, x1 = seg == 0 ? xa1 : xb1;
      for (int xu = x0; xu <= x1; ++xu) {
        int x = xu % B.lx;
        x = x < 0 ? x + B.lx : x;
        double dn[3];
        int kn;
        minimage(B, (double)x - Rn[0], (double)y - Rn[1], (double)z - Rn[2], dn[0], dn[1], dn[2], kn);
        if (kn != k) continue;  // reached through another image box
        const bool in_new = dn[0] * dn[0] + dn[1] * dn[1] + dn[2] * dn[2] < a2;
        double dd0, dd1, dd2;
        int ko;
        minimage(bold, (double)x - Ro[0], (double)y - Ro[1], (double)z - Ro[2], dd0, dd1, dd2, ko);
        const bool in_old = dd0 * dd0 + dd1 * dd1 + dd2 * dd2 < a2;
        const int64_t node = x + (int64_t)B.lx * (y + (int64_t)B.ly * z);
        if (PHASE == 1 && in_new && !in_old) {
          const int32_t v = atomicCAS(&A.own[node], -1, p);
          if (v == -1) {
            // covered: the node's fluid mass and momentum go to the sphere
            double rho = 0, j0 = 0, j1 = 0, j2 = 0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
              const double fv = wq(q) * A.rho0 +
                                (double)Store<ST>::ld((const ST *)A.f + (size_t)q * A.plane, node, q, A.h16);
              rho += fv; j0 += fv * cx(q); j1 += fv * cy(q); j2 += fv * cz(q);
            }
            j0 -= rho * kn * B.ule;
            acc[0] += j0; acc[1] += j1; acc[2] += j2;
            acc[3] += dn[1] * j2 - dn[2] * j1;
            acc[4] += dn[2] * j0 - dn[0] * j2;
            acc[5] += dn[0] * j1 - dn[1] * j0;
            acc[6] += rho;
          } else if (v != p) {
            if (inside_new(A, bnew, v, x, y, z)) {  // both spheres hold the node: overlap
              atomicMin(&A.own[node], p);
              atomicOr(A.flags, 1);
            } else if (atomicCAS(&A.own[node], v, p) != v) {  // v left it; a third claim is an overlap
              atomicMin(&A.own[node], p);
              atomicOr(A.flags, 1);
            }
          }
        }
        if (PHASE == 2 && in_old && !in_new && A.own[node] == p) {
          // released: equilibrium at rho0 and the surface velocity of the moved sphere
          A.own[node] = -1;
          const double *W = &A.W[3 * p];
          const double ub0 = A.U[3 * p] + (W[1] * dn[2] - W[2] * dn[1]);
          const double ub1 = A.U[3 * p + 1] + (W[2] * dn[0] - W[0] * dn[2]);
          const double ub2 = A.U[3 * p + 2] + (W[0] * dn[1] - W[1] * dn[0]);
          const double ux = ub0 + kn * B.ule;
          const double uu = ux * ux + ub1 * ub1 + ub2 * ub2;
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            const double cu = cx(q) * ux + cy(q) * ub1 + cz(q) * ub2;
            const double dv = wq(q) * A.rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
            Store<ST>::st((ST *)A.f + (size_t)q * A.plane, node, (CT)dv, q, A.h16);
          }
          const double j0 = A.rho0 * ub0, j1 = A.rho0 * ub1, j2 = A.rho0 * ub2;
          acc[0] -= j0; acc[1] -= j1; acc[2] -= j2;
          acc[3] -= dn[1] * j2 - dn[2] * j1;
          acc[4] -= dn[2] * j0 - dn[0] * j2;
          acc[5] -= dn[0] * j1 - dn[1] * j0;
          acc[6] -= A.rho0;
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 7; ++c) acc[c] = wsum(acc[c]);
  if (lane != 0) return;
  double *dp = &A.dp[(size_t)p * 8];
  if (PHASE == 1) {
    for (int c = 0; c < 7; ++c) dp[c] = acc[c];
    return;
  }
  for (int c = 0; c < 7; ++c) dp[c] += acc[c];
  if (A.wmem && A.wmem[p] > 0) return;  // prescribed motion: the impulses load the wall
  double U[3], W[3];
  for (int c = 0; c < 3; ++c) {
    U[c] = A.U[3 * p + c] + dp[c] / A.m[p];
    W[c] = A.W[3 * p + c] + dp[3 + c] / A.I[p];
  }
  if (A.quasi2d) { U[2] = 0.0; W[0] = 0.0; W[1] = 0.0; }
  for (int c = 0; c < 3; ++c) { A.Uw[3 * p + c] = U[c]; A.Ww[3 * p + c] = W[c]; }
}

template <class ST, int PHASE>
__global__ __launch_bounds__(64) void k_map_update(MapArgs A) { map_update_wg<ST, PHASE>(A, (int)blockIdx.x); }
template <class ST, int PHASE>
__global__ __launch_bounds__(64) void k_map_update_m(const MapArgs *__restrict__ tab, const int32_t *__restrict__ pre,
                                                     int nj) {
  SUSP_MULTI_BODY(MapArgs, (map_update_wg<ST, PHASE>));
}

hipError_t launch_map_update(Sim *s, const Box &box, int phase) {
  MapArgs A;
  A.R = s->R[s->pcur]; A.U = s->U[s->pcur]; A.W = s->W[s->pcur];
  A.R0 = s->R0; A.amap = s->amap; A.m = s->m; A.I = s->I;
  A.Uw = s->U[s->pcur]; A.Ww = s->W[s->pcur];
  A.own = s->own;
  A.f = s->f[s->cur]; A.plane = s->plane;
  A.b = box; A.clk = s->clk;
  A.rho0 = s->rho0; A.quasi2d = s->quasi2d;
  A.dp = s->dp; A.flags = s->flags;
  A.h16 = s->h16;
  A.wmem = s->boundary == 1 ? s->wmem : nullptr;
  if (s->n == 0) return hipSuccess;
  const unsigned g = s->n;
  if (phase == 1) {
    if (s->precision == 0) return dispatch(s, k_map_update<double, 1>, k_map_update_m<double, 1>, g, 64, A);
    if (s->precision == 1) return dispatch(s, k_map_update<float, 1>, k_map_update_m<float, 1>, g, 64, A);
    return dispatch(s, k_map_update<__half, 1>, k_map_update_m<__half, 1>, g, 64, A);
  }
  if (s->precision == 0) return dispatch(s, k_map_update<double, 2>, k_map_update_m<double, 2>, g, 64, A);
  if (s->precision == 1) return dispatch(s, k_map_update<float, 2>, k_map_update_m<float, 2>, g, 64, A);
  return dispatch(s, k_map_update<__half, 2>, k_map_update_m<__half, 2>, g, 64, A);
}

// ---------------------------------------------------------------------------------------
// Stress reduction in one launch.  Block b sums a contiguous slice of the lattice-brick
// partials and of the spheres into part[b][RED_W]; the block that finishes last (a counter in
// the flags block, reset by that block) adds the slices in order and updates the accumulators.
// part: pineq 6 | hydro stresslet 6 | pair 18 | ledger 1 | fluid mass deviation 1 | fluid nodes 1
constexpr int RED_N = 33;
struct ReduceArgs {
  const double *pin, *hyd, *pst, *dp;
  int nblk, n;
  double *part, *acc;
  // cf: fluid stress factor -(1 - 1/(2 tau)) / V; cfb the same with tau_bulk for the trace
  // (multi-eigenvalue collision, split = 1)
  double cf, cfb, invV, invns, rho0, mass_tol;
  int split, has_particles;
  const Clock *clk;
  int32_t *flags;
  int nred;  // work-groups of the reduction (<= RED_BLOCKS; one slice each)
};

// The fluid mass plus the ledger is conserved by the method (bounce-back links pair up along
// every lattice line, covered and released nodes pass through the ledger); a drift above
// mass_tol from its value at the first step reduced raises FL_MASS.
//
// The slices in a fixed order: 7 groups of threads per component take every 7th slice, then
// the groups in order; a thread per stress component updates the accumulators.
constexpr int RED_G = 7;  // RED_G * RED_N <= 256
__device__ void reduce_final(const ReduceArgs &A) {
  __shared__ double gs[RED_G][RED_N];
  __shared__ double v[RED_N], sig[30];
  const int t = threadIdx.x;
  if (t < RED_G * RED_N) {
    const int g = t / RED_N, c = t - g * RED_N;
    double x = 0.0;
#pragma unroll 4
    for (int b = g; b < A.nred; b += RED_G) x += A.part[(size_t)b * RED_W + c];
    gs[g][c] = x;
  }
  __syncthreads();
  if (t < RED_N) {
    double x = gs[0][t];
    for (int g = 1; g < RED_G; ++g) x += gs[g][t];
    v[t] = x;
  }
  __syncthreads();
  double *acc = A.acc;
  if (t < 30) {  // fluid, hydrodynamic, lubrication, contact, DLVO: six components each
    const int kk = t / 6, k = t - 6 * kk;
    const double t3 = (v[0] + v[1] + v[2]) / 3.0;
    double x;
    if (kk == 0) x = (A.split && k < 3) ? A.cf * (v[k] - t3) + A.cfb * t3 : A.cf * v[k];
    else if (kk == 1) x = A.has_particles ? v[6 + k] * A.invV : 0.0;
    else x = v[6 * kk + k] * A.invV * A.invns;
    sig[t] = x;
    acc[t] = x;
    acc[30 + t] += x;
  }
  __syncthreads();
  if (t != 0) return;
  double sxy = 0;
  for (int k = 0; k < 5; ++k) sxy += sig[6 * k + 3];
  acc[60] += 1.0;
  const ClockEntry &ce = A.clk->cur;
  if (ce.gphase) { acc[61] += sxy * ce.gcos; acc[62] += sxy * ce.gsin; acc[63] += 1.0; }
  // the lattice kernel measured the fluid mass before this step's map update, so it pairs
  // with the ledger as it stood before this step's covers and releases
  const double mass = v[31] + v[32] * A.rho0;
  acc[65] = mass;
  if (acc[67] == 0.0) {
    acc[66] = mass + acc[64];
    acc[67] = 1.0;
  } else if (!(fabs(mass + acc[64] - acc[66]) <= A.mass_tol)) {
    atomicOr(A.flags, FL_MASS);
  }
  acc[68] = acc[64];  // the ledger that pairs with this step's fluid mass
  acc[64] += v[30];
}

__device__ __forceinline__ void reduce_wg(const ReduceArgs &A, const int bid) {
  double v[RED_N];
  for (int c = 0; c < RED_N; ++c) v[c] = 0.0;
  const int b = bid;
  const int pb0 = (int)((int64_t)A.nblk * b / A.nred), pb1 = (int)((int64_t)A.nblk * (b + 1) / A.nred);
  for (int t = pb0 + threadIdx.x; t < pb1; t += blockDim.x) {
    for (int c = 0; c < 6; ++c) v[c] += A.pin[(size_t)t * 8 + c];
    v[31] += A.pin[(size_t)t * 8 + 6];
    v[32] += A.pin[(size_t)t * 8 + 7];
  }
  const int s0 = (int)((int64_t)A.n * b / A.nred), s1 = (int)((int64_t)A.n * (b + 1) / A.nred);
  for (int p = s0 + threadIdx.x; p < s1; p += blockDim.x) {
    for (int c = 0; c < 6; ++c) v[6 + c] += A.hyd[(size_t)p * HYD + 6 + c];
    for (int c = 0; c < PST; ++c) v[12 + c] += A.pst[(size_t)p * PST + c];
    v[30] += A.dp[(size_t)p * 8 + 6];
  }
  // each wave's lanes by a fixed butterfly, then the four waves in order, a thread per component
  __shared__ double sh[RED_N][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < RED_N; ++c) {
    const double x = wsum(v[c]);
    if (lane == 0) sh[c][wv] = x;
  }
  __syncthreads();
  if (threadIdx.x < RED_N) {
    const int c = threadIdx.x;
    A.part[(size_t)b * RED_W + c] = (sh[c][0] + sh[c][1]) + (sh[c][2] + sh[c][3]);
    __threadfence();  // the slice is visible before the count
  }
  __syncthreads();
  __shared__ int last;
  if (threadIdx.x == 0) last = atomicAdd(A.flags + FL_REDCNT, 1) == A.nred - 1;
  __syncthreads();
  if (!last) return;  // the whole block
  __threadfence();  // every slice visible to this block's loads
  if (threadIdx.x == 0) A.flags[FL_REDCNT] = 0;  // for the next step's reduction
  reduce_final(A);
}
__global__ __launch_bounds__(256) void k_reduce(ReduceArgs A) { reduce_wg(A, (int)blockIdx.x); }
__global__ __launch_bounds__(256) void k_reduce_m(const ReduceArgs *__restrict__ tab, const int32_t *__restrict__ pre,
                                                  int nj) {
  SUSP_MULTI_BODY(ReduceArgs, reduce_wg);
}

hipError_t launch_stress(Sim *s) {
  ReduceArgs A;
  A.pin = s->pin; A.hyd = s->hyd[s->hcur]; A.pst = s->pst; A.dp = s->dp;
  A.nblk = s->nbricks; A.n = s->n;
  A.part = s->acc + ACC_PART; A.acc = s->acc;
  const double V = (double)s->lx * s->ly * s->lz;
  A.cf = -(1.0 - 0.5 / s->tau) / V;
  A.cfb = -(1.0 - 0.5 / s->tau_bulk) / V;
  A.invV = 1.0 / V;
  A.invns = 1.0 / (double)s->n_sub;
  A.rho0 = s->rho0;
  A.mass_tol = MASS_TOL * V * s->rho0;
  A.split = s->collision;
  A.has_particles = s->n > 0 ? 1 : 0;
  A.clk = s->clk;
  A.flags = s->flags;
  // one work-group per 512 bricks or spheres: each one's fence writes back its L2, so the
  // count is kept to what the data needs
  const int64_t items = s->nbricks > s->n ? s->nbricks : s->n;
  A.nred = (int)((items + 511) / 512);
  A.nred = A.nred < 1 ? 1 : (A.nred > RED_BLOCKS ? RED_BLOCKS : A.nred);
  return dispatch(s, k_reduce, k_reduce_m, (unsigned)A.nred, 256, A);
}

// ---------------------------------------------------------------------------------------
// Contact statistics.  Per step: k_cstat_part sums the recorded contacts of 256 spheres per
// work-group, for one orientation bin (count, sum F_nor, sum F_tan) or, in the last bin
// index, over all contacts (count, sum F_nor, and the four in-plane components of
// [F_nor n - F_tan t] (x) n, the integrand of eqs. 26-27); k_cstat_acc adds the chunks in
// order to the running sums together with the step's total stress.  Fixed orders
// throughout, so the statistics are bitwise reproducible.
struct CstatArgs {
  const int32_t *cnt, *cflag;
  const double *rec;
  double *part;
  int n, nb, chunks;
};

// Orientation bin of the in-plane direction (nx, ny): the angle folded into [0, pi) (both
// senses are one orientation), in FP64, nb equal bins.
__device__ inline int orient_bin(double nx, double ny, int nb) {
  const double PI = 3.14159265358979323846;
  double ox = nx, oy = ny;
  if (oy < 0.0 || (oy == 0.0 && ox < 0.0)) { ox = -ox; oy = -oy; }
  const double th = atan2(oy, ox);
  const int bin = (int)(th * (double)nb / PI);
  return bin < 0 ? 0 : (bin > nb - 1 ? nb - 1 : bin);
}

__global__ __launch_bounds__(256) void k_cstat_part(CstatArgs A) {
  __shared__ double red[6][256];
  const int b = blockIdx.x / A.chunks, k = blockIdx.x % A.chunks;
  const int t = threadIdx.x, i = k * 256 + t;
  double v[6] = {0, 0, 0, 0, 0, 0};
  if (i < A.n) {
    const int c = A.cnt[i];
    for (int u = 0; u < c; ++u) {
      const size_t e = (size_t)i * NCAP + u;
      if (A.cflag[e] == 0) continue;
      const double nx = A.rec[4 * e], ny = A.rec[4 * e + 1];
      if (b < A.nb && orient_bin(nx, ny, A.nb) != b) continue;
      const double fn = A.rec[4 * e + 2], ft = A.rec[4 * e + 3];
      v[0] += 1.0;
      v[1] += fn;
      if (b < A.nb) {
        v[2] += ft;
      } else {
        const double vx = fn * nx - ft * (-ny), vy = fn * ny - ft * nx;
        v[2] += vx * nx; v[3] += vx * ny; v[4] += vy * nx; v[5] += vy * ny;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) red[c][t] = v[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
      for (int c = 0; c < 6; ++c) red[c][t] += red[c][t + w];
    __syncthreads();
  }
  if (t < 6) A.part[(size_t)blockIdx.x * 6 + t] = red[t][0];
}

// one wave per bin (and the totals): lane l adds chunks l, l + 64, ... in order, then a fixed
// butterfly over the lanes; acc[0..29] holds this step's stress parts
__global__ __launch_bounds__(64) void k_cstat_acc(const double *part, double *cacc, const double *acc, int nb,
                                                  int chunks) {
  const int b = blockIdx.x, l = threadIdx.x;
  for (int c = 0; c < 6; ++c) {
    double x = 0.0;
    for (int k = l; k < chunks; k += 64) x += part[((size_t)b * chunks + k) * 6 + c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (l == 0) cacc[b * 6 + c] += x;
  }
  if (b == nb && l == 0) {
    double *sg = cacc + (nb + 1) * 6;
    for (int c = 0; c < 6; ++c) sg[c] += acc[c] + acc[6 + c] + acc[12 + c] + acc[18 + c] + acc[24 + c];
    sg[6] += 1.0;
  }
}

hipError_t launch_contact_sample(Sim *s) {
  if (s->cbins <= 0) return hipSuccess;
  SUSP_NO_COLLECT(s);
  if (s->n > 0) {
    CstatArgs A;
    A.cnt = s->ncnt[s->lcur]; A.cflag = s->cflag; A.rec = s->crec; A.part = s->cpart;
    A.n = s->n; A.nb = s->cbins; A.chunks = s->cchunks;
    hipLaunchKernelGGL(k_cstat_part, dim3((s->cbins + 1) * s->cchunks), dim3(256), 0, s->stream, A);
  } else {
    hipError_t e = launch_fill_f64(s->cpart, (size_t)(s->cbins + 1) * s->cchunks * 6, 0.0, s->stream);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_cstat_acc, dim3(s->cbins + 1), dim3(64), 0, s->stream, s->cpart, s->cacc, s->acc,
                     s->cbins, s->cchunks);
  return hipGetLastError();
}

// Eigenvalues of a symmetric 3x3 matrix (xx yy zz xy xz yz), descending: the trigonometric
// solution of the characteristic cubic (Smith, Commun. ACM 4, 168 (1961)).
__device__ inline void sym3_eig(const double m[6], double ev[3]) {
  const double PI = 3.14159265358979323846;
  const double p1 = m[3] * m[3] + m[4] * m[4] + m[5] * m[5];
  const double q = (m[0] + m[1] + m[2]) / 3.0;
  if (p1 == 0.0) {
    ev[0] = m[0]; ev[1] = m[1]; ev[2] = m[2];
  } else {
    const double a = m[0] - q, b = m[1] - q, c = m[2] - q;
    const double p = sqrt((a * a + b * b + c * c + 2.0 * p1) / 6.0);
    const double ip = 1.0 / p;
    const double B0 = a * ip, B1 = b * ip, B2 = c * ip, B3 = m[3] * ip, B4 = m[4] * ip, B5 = m[5] * ip;
    // det(B) / 2 with B = (A - q I) / p
    double r = 0.5 * (B0 * (B1 * B2 - B5 * B5) - B3 * (B3 * B2 - B5 * B4) + B4 * (B3 * B5 - B1 * B4));
    r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
    const double phi = acos(r) / 3.0;
    ev[0] = q + 2.0 * p * cos(phi);
    ev[2] = q + 2.0 * p * cos(phi + 2.0 * PI / 3.0);
    ev[1] = 3.0 * q - ev[0] - ev[2];
  }
  for (int i = 0; i < 3; ++i)
    for (int k = i + 1; k < 3; ++k)
      if (ev[k] > ev[i]) { const double x = ev[i]; ev[i] = ev[k]; ev[k] = x; }
}

// Read-out: the distributions of eqs. 19-23 per bin, <F_nor>, Z, the stress of eq. 27 (3D) or
// eq. 26 (monolayer, per unit volume), Delta lambda / P of the mean total stress; then the
// running sums are cleared.  One work-group of 256 threads.
__global__ __launch_bounds__(256) void k_cstat_final(double *cacc, double *out, int nb, int n, double amean,
                                                     double frac, int quasi2d, double lz) {
  const double PI = 3.14159265358979323846;
  const double *tot = cacc + nb * 6;
  const double *sg = cacc + (nb + 1) * 6;
  const double nc = tot[0];
  const double fmean = nc > 0.0 ? tot[1] / nc : 0.0;
  const double dth = PI / (double)nb;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    const double c = cacc[b * 6];
    const double rho = nc > 0.0 ? c / (nc * dth) : 0.0;
    const double fnor = c > 0.0 ? cacc[b * 6 + 1] / c : 0.0;
    const double ftan = c > 0.0 ? cacc[b * 6 + 2] / c : 0.0;
    const double xn = fmean != 0.0 ? fnor / fmean : 0.0;
    const double xt = fmean != 0.0 ? ftan / fmean : 0.0;
    out[b] = rho;
    out[nb + b] = xn;
    out[2 * nb + b] = xt;
    out[3 * nb + b] = rho * xn;
    out[4 * nb + b] = rho * xt;
  }
  if (threadIdx.x == 0) {
    double *sm = out + 5 * nb;
    const double samples = sg[6];
    const double Z = (n > 0 && samples > 0.0) ? 2.0 * nc / ((double)n * samples) : 0.0;
    double C = 0.0;
    if (amean > 0.0)
      C = quasi2d ? frac * Z / (PI * amean) / lz : 3.0 * frac * Z / (4.0 * PI * amean * amean);
    double M[6];
    for (int c = 0; c < 6; ++c) M[c] = samples > 0.0 ? sg[c] / samples : 0.0;
    double dl, pr;
    if (quasi2d) {
      const double mid = 0.5 * (M[0] + M[1]);
      dl = 2.0 * sqrt(0.25 * (M[0] - M[1]) * (M[0] - M[1]) + M[3] * M[3]);
      pr = -mid;
    } else {
      double ev[3];
      sym3_eig(M, ev);
      dl = ev[0] - ev[2];
      pr = -(ev[0] + ev[1] + ev[2]) / 3.0;
    }
    sm[0] = samples;
    sm[1] = samples > 0.0 ? nc / samples : 0.0;
    sm[2] = Z;
    sm[3] = fmean;
    for (int k = 0; k < 4; ++k) sm[4 + k] = nc > 0.0 ? C * (tot[2 + k] / nc) : 0.0;
    sm[8] = dl;
    sm[9] = pr;
    sm[10] = pr != 0.0 ? dl / pr : 0.0;
    sm[11] = frac;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < (nb + 1) * 6 + 8; k += blockDim.x) cacc[k] = 0.0;
}

// Force of the suspension on the bottom and top walls this step: the flat walls' block sums
// in block order, then each wall sphere's force and its cover/uncover impulses in sphere
// order (fixed orders), added to the running sums.  One work-group.
__global__ __launch_bounds__(256) void k_wall_force(const double *wpart, int nblk, const int32_t *wmem,
                                                    const double *wfs, const double *dp, int n,
                                                    double *wacc) {
  __shared__ double red[6][256];
  const int t = threadIdx.x;
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int b = t; b < nblk; b += 256)
    for (int c = 0; c < 6; ++c) v[c] += wpart[(size_t)b * 6 + c];
  for (int i = t; i < n; i += 256) {
    const int m = wmem[i];
    if (m <= 0) continue;
    for (int c = 0; c < 3; ++c) v[3 * (m - 1) + c] += wfs[3 * i + c] + dp[(size_t)i * 8 + c];
  }
  for (int c = 0; c < 6; ++c) red[c][t] = v[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
      for (int c = 0; c < 6; ++c) red[c][t] += red[c][t + w];
    __syncthreads();
  }
  if (t < 6) wacc[t] += red[t][0];
  if (t == 0) wacc[6] += 1.0;
}

hipError_t launch_wall_force(Sim *s) {
  SUSP_NO_COLLECT(s);
  const int nblk = (2 * s->lx * s->lz + 255) / 256;
  hipLaunchKernelGGL(k_wall_force, dim3(1), dim3(256), 0, s->stream, s->wpart, nblk, s->wmem, s->wfs, s->dp,
                     s->n, s->wacc);
  return hipGetLastError();
}

// The read-out into out[5 nb + 12] (the simulation's staging, or a caller's).
hipError_t launch_contact_final(Sim *s, double *out) {
  hipLaunchKernelGGL(k_cstat_final, dim3(1), dim3(256), 0, s->stream, s->cacc, out, s->cbins, s->n,
                     s->cgeo[0], s->cgeo[1], s->quasi2d, (double)s->lz);
  return hipGetLastError();
}

}  // namespace susp
