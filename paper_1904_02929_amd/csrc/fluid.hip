// fluid.hip -- lattice-Boltzmann kernels for gfx950.
//
//  k_lattice  links and stream of one 64 x 4 x 4 brick per work-group (the default with spheres)
//  k_links    the step's links, (fluid node, sphere, directions) per brick in LDS, their
//             moving bounce-back and the exchanged momentum summed per sphere (App. A eqs. 6-10)
//  k_stream   pull-stream + collision + fluid stress partials (App. A eqs. 3-5), one thread
//             per fluid node, x fastest
//  k_ghost_raster, k_ghost_values  Lees-Edwards ghost planes y=-1 and y=ly: the owner of each
//             ghost point by the geometric test against the spheres' images, else linear
//             interpolation of the Galilean-corrected post-collision row shifted by the offset
//             (Wagner & Pagonabarraga).
//  helpers    equilibrium fill, FP64 <-> storage conversion, link enumeration.
#include "susp_impl.h"

#include <algorithm>
#include <type_traits>

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
// The lattice step of App. A in two kernels.
//   k_links     the links of the step: for every fluid node and every sphere that some of its
//               pull sources x - c_q belong to, one entry (node, sphere, those directions q),
//               listed per brick in LDS (across the sliding plane the source is a ghost
//               point, whose owner k_ghost_raster decided against the sphere images); per entry
//               the bounce-back of eq. 7 on those links, written where the pull will read
//               it, and the momentum each link exchanges (eq. 6) summed into the sphere's
//               force, torque and stresslet (eqs. 9, 10).
//   k_stream    per fluid node: pull (eq. 3; a link now reads its prepared value), collision
//               (eqs. 4, 5) on the deviations d_q = n_q - w_q rho0, the fluid stress and mass
//               partials; rows are stored whole, a solid node as the rest state.
constexpr int TX = 64;      // brick width: one wave per 64-node row segment
constexpr int TS = 32;      // per-work-group table slots of k_links (spheres seen by its entries)
constexpr int NPIN = 8;     // per-brick partials: Pi^neq xx yy zz xy xz yz, sum (rho - rho0), fluid nodes
constexpr int LMAXS = 6;    // spheres one node can link to

// Per-sphere sums without a summation order.  A value v enters as two integers, hi =
// rint(v 2^FXH) and lo = rint((v - hi 2^-FXH) 2^FXL), added with 64-bit integer atomics;
// integer addition is associative, so the total is the same bits whatever order the
// additions take (any brick shape, any interleaving of the work-groups).  The split is
// exact (|lo| <= 2^(FXL-FXH-1)); hi is formed as a 32-bit integer and lo by adding 1.5 2^52,
// which puts the rounded integer (ties to even, as rint) in the low mantissa bits, so one
// term needs |v| < 2^(31-FXH) (the link sums of one node and sphere are far below); a sphere
// may take up to 2^15 additions per step before lo can overflow; the rounding of lo costs
// 2^-69 per term.
__device__ inline void fx_split(double v, unsigned long long &h, unsigned long long &l) {
  constexpr double M = 6755399441055744.0;  // 1.5 2^52
  const double hv = rint(ldexp(v, FXH));
  const double tl = ldexp(v - ldexp(hv, -FXH), FXL) + M;  // the remainder is exact
  h = (unsigned long long)(long long)(int)hv;
  l = (unsigned long long)(__double_as_longlong(tl) - __double_as_longlong(M));
}
__device__ inline void fx_add(unsigned long long *dst, double v) {
  unsigned long long h, l;
  fx_split(v, h, l);
  atomicAdd(dst, h);
  atomicAdd(dst + 1, l);
}
// the same into a work-group's LDS table entry (an LDS-typed pointer, so that the additions
// are LDS atomics even where the code beside them adds into global memory)
typedef __attribute__((address_space(3))) unsigned long long lds_u64;
__device__ inline lds_u64 *as_lds(unsigned long long *p) { return (lds_u64 *)p; }
__device__ inline void fx_lds(lds_u64 *e, double v) {
  unsigned long long h, l;
  fx_split(v, h, l);
  __hip_atomic_fetch_add(e, h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  __hip_atomic_fetch_add(e + 1, l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}


// c_q . (ax, ay, az) for a compile-time q, summed x, y, z in order without the zero terms.
template <class T> __device__ inline T cdot(int q, T ax, T ay, T az) {
  T s = 0;
  bool first = true;
  if (cx(q) != 0) { s = cx(q) > 0 ? ax : -ax; first = false; }
  if (cy(q) != 0) { const T v = cy(q) > 0 ? ay : -ay; s = first ? v : s + v; first = false; }
  if (cz(q) != 0) { const T v = cz(q) > 0 ? az : -az; s = first ? v : s + v; }
  return s;
}
// acc += c * v for c in {-1, 0, 1} known at compile time
template <class T> __device__ inline void addc(T &acc, int c, T v) {
  if (c > 0) acc += v;
  else if (c < 0) acc -= v;
}

// Link sums over the 9 opposite pairs: coefficient kind sel (0 c_x, 1 c_y, 2 c_z, 3 c_x c_y,
// 4 c_x c_z, 5 c_y c_z) of direction q, and the first pair where it is nonzero.
__host__ __device__ constexpr int pair_coef(int sel, int q) {
  return sel == 0 ? cx(q) : sel == 1 ? cy(q) : sel == 2 ? cz(q)
       : sel == 3 ? cx(q) * cy(q) : sel == 4 ? cx(q) * cz(q) : cy(q) * cz(q);
}
__host__ __device__ constexpr int first_pair(int sel) {
  int f = 9;
  for (int pi = 8; pi >= 0; --pi)
    if (pair_coef(sel, 2 * pi + 1) != 0) f = pi;
  return f;
}
// acc += c * v (c in {-1, 0, 1}, compile time) for pair pi, or acc = c * v at the first pair
// of its kind
__device__ inline void acc_pair(double &acc, int pi, int sel, int c, double v) {
  const bool first = pi == first_pair(sel);
  if (c > 0) acc = first ? v : acc + v;
  else if (c < 0) acc = first ? -v : acc - v;
}
// 1/x: the hardware reciprocal in FP32 (within 1 ulp), a division in FP64
__device__ inline float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double recip(double x) { return 1.0 / x; }
__device__ inline float fmaT(float a, float b, float c) { return fmaf(a, b, c); }
__device__ inline double fmaT(double a, double b, double c) { return fma(a, b, c); }

// Population access through a buffer resource over a whole array (< 4 GiB): the 32-bit
// byte offset is the sum of a uniform part (plane and row, scalar registers) and the lane's
// x; an offset past the array reads 0 and writes nothing.
__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
template <class ST> struct RowIO;
template <> struct RowIO<double> {
  __device__ static double ld(__amdgpu_buffer_rsrc_t r, uint32_t off, int, H16) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  }
  __device__ static void st(__amdgpu_buffer_rsrc_t r, uint32_t off, double v, int, H16) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
  }
  // a store no later kernel of the step reads (non-temporal: streamed past the caches)
  __device__ static void st_stream(__amdgpu_buffer_rsrc_t r, uint32_t off, double v, int, H16) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 2);
  }
};
template <> struct RowIO<float> {
  __device__ static float ld(__amdgpu_buffer_rsrc_t r, uint32_t off, int, H16) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  }
  __device__ static void st(__amdgpu_buffer_rsrc_t r, uint32_t off, float v, int, H16) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 0);
  }
  __device__ static void st_stream(__amdgpu_buffer_rsrc_t r, uint32_t off, float v, int, H16) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 2);
  }
};
// FP16 storage: same scaling as Store<__half>
template <> struct RowIO<__half> {
  __device__ static float ld(__amdgpu_buffer_rsrc_t r, uint32_t off, int q, H16 h) {
    const unsigned short b = __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
    return __half2float(__builtin_bit_cast(__half, b)) * ((float)wq(q) * h.dn);
  }
  __device__ static void st(__amdgpu_buffer_rsrc_t r, uint32_t off, float v, int q, H16 h) {
    const __half hv = __float2half_rn(v * ((float)(1.0 / wq(q)) * h.up));
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, hv), r, off, 0, 0);
  }
  __device__ static void st_stream(__amdgpu_buffer_rsrc_t r, uint32_t off, float v, int q, H16 h) {
    const __half hv = __float2half_rn(v * ((float)(1.0 / wq(q)) * h.up));
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, hv), r, off, 0, 2);
  }
  // the lattice kernel keeps the 16 stored bits in a float register until the value is
  // used (a step later), so that the conversion does not wait for the load
  __device__ static float raw(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float, (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0));
  }
  __device__ static float dec(float v, int q, H16 h) {
    const unsigned short b = (unsigned short)__builtin_bit_cast(uint32_t, v);
    return __half2float(__builtin_bit_cast(__half, b)) * ((float)wq(q) * h.dn);
  }
};



// Minimum image of a node X against a sphere centre R, both inside the box (the particle
// update keeps R in [0, L)): one sliding-plane crossing in y, then one wrap in x (after the
// image's shift s) and z.  Agrees with minimage except exactly half a period apart; either
// way the node's links are then checked against the image it gives (links_in_image).
__device__ inline void node_image(const Box &b, double ilx, double ilz, double dx, double dy, double dz,
                                  double &ox, double &oy, double &oz, int &k) {
  k = dy > 0.5 * b.Ly ? 1 : (dy < -0.5 * b.Ly ? -1 : 0);
  dy -= k * b.Ly;
  dx -= k * b.s;
  ox = dx - b.Lx * rint(dx * ilx);
  oy = dy;
  oz = dz - b.Lz * rint(dz * ilz);
}

// Masks (bit q) of the D3Q19 directions whose component along axis (0 x, 1 y, 2 z) is sgn.
__host__ __device__ constexpr uint32_t dir_mask(int axis, int sgn) {
  uint32_t m = 0;
  for (int q = 1; q < NQ; ++q)
    if ((axis == 0 ? cx(q) : axis == 1 ? cy(q) : cz(q)) == sgn) m |= 1u << q;
  return m;
}
// Whether every link in m ends in the image whose centre gives the node's lever D: for each
// linked q, each component of D - c_q (the solid end X - c_q minus that centre) lies inside the
// half period, so the minimum image of the solid end is that image.  The node's links can then
// be summed per node (eq. 8: u_b . c_q = u(X) . c_q, and each lever is D - c_q / 2).
__device__ inline bool links_in_image(uint32_t m, const Box &bx, double Dx, double Dy, double Dz) {
  const double hx = 0.5 * bx.Lx - 1e-6, hy = 0.5 * bx.Ly - 1e-6, hz = 0.5 * bx.Lz - 1e-6;
  constexpr uint32_t XP = dir_mask(0, 1), XN = dir_mask(0, -1), YP = dir_mask(1, 1), YN = dir_mask(1, -1),
                     ZP = dir_mask(2, 1), ZN = dir_mask(2, -1);
  bool ok = true;
  if (m & XP) ok = ok && fabs(Dx - 1.0) <= hx;
  if (m & XN) ok = ok && fabs(Dx + 1.0) <= hx;
  if (m & ~(XP | XN)) ok = ok && fabs(Dx) <= hx;
  if (m & YP) ok = ok && fabs(Dy - 1.0) <= hy;
  if (m & YN) ok = ok && fabs(Dy + 1.0) <= hy;
  if (m & ~(YP | YN)) ok = ok && fabs(Dy) <= hy;
  if (m & ZP) ok = ok && fabs(Dz - 1.0) <= hz;
  if (m & ZN) ok = ok && fabs(Dz + 1.0) <= hz;
  if (m & ~(ZP | ZN)) ok = ok && fabs(Dz) <= hz;
  return ok;
}

// A wave-uniform value the compiler must treat as unknown at this point: what derives from
// it (row and plane offsets) is formed where it is used instead of being hoisted out of the
// loops into dozens of live scalar registers.
__device__ inline int opaque_uniform(int v) {
  v = __builtin_amdgcn_readfirstlane(v);
  asm volatile("" : "+s"(v));
  return v;
}


// ---- k_links: a work-group per brick of LBX x LBY x LBZ nodes, the bricks dealt to the 8
// XCDs in contiguous ranges (neighbouring bricks share an L2).
//  list    wave w takes row y0 + w through the brick's z-slices, one lane per node: the owners
//          of its 18 pull sources x - c_q (all slices' loads issued together) and the
//          distinct spheres among them, one entry (sphere, node, link directions) each in an
//          LDS list.  Where all linked sources belong to one sphere (most nodes) the largest
//          and smallest owner agree; otherwise the spheres are taken in decreasing id.  The
//          list order does not matter: each entry's sums are its own and the per-sphere
//          totals are integers.
//  table   the spheres of the entries get slots in an LDS table (open addressing); the lane
//          that claims a slot stages the sphere's centre and velocities in LDS.
//  links   one lane per entry.  With lever r_b - R = D - c_q/2 (D = node minus sphere
//          centre, minimum image) the surface velocity along a link is u_b . c_q = u(X) . c_q,
//          because (W x c) . c = 0: one rigid-body velocity per entry, and per link
//            corr = -6 w_q rho0 u(X) . c_q,  n_q = n*_qbar - corr,  m = 2 n*_qbar - corr
//          (the rest part 2 w_q rho0 of the exchanged momentum left out: the sums are
//          measured from the rest state).  n_q goes to the link values at the end of the
//          population buffer, where k_stream's pull takes it (see the record below).
//          corr, m and the entry's sums F = -sum m c_q, T = D x F, S = sym(D (x) F)
//          + 1/2 sum m c_q c_q are formed in FP64 (a sphere's sums cancel over its surface
//          to a small remainder); a convex sphere links a node through at most one of two
//          opposite directions, so they run over the 9 opposite pairs.  The entry's sums go
//          into the table as fixed-point integers (order-free, see fx_add), and at the end
//          into the spheres' sums.
// Link values: each brick owns a block of LINK_CAP values per node; the list phase gives each
// 64-node row of the brick a run of it (one value per link of its nodes, in node order and
// direction order within a node, placed by an LDS counter) and each node a record: its link
// directions, whether it is solid, and the offset of its first value in the row's run.  The
// writes are contiguous, and k_stream reads a node's values next to each other.
constexpr int LBX = 64, LBY = 4, LBZ = 4;  // k_links brick: one wave per row, through the z-slices
constexpr int LCAP = 2048;                  // LDS list: 2 entries per node of the brick
struct LinksArgs {
  void *f;                 // the step's input populations, then the link values after them
  size_t plane;
  uint32_t pop_bytes;
  uint32_t ow_bytes;  // the owner map and the ghost owner planes after it, as one array
  int goff;           // elements from the owner map's start to the ghost planes
  const int32_t *own;
  const double *R, *U, *W;
  unsigned long long *hacc;  // [n][HYD][2]
  int32_t *flags;
  uint32_t *lrec;            // [nodes] link records (null: kept in LDS only, for k_lattice)
  int32_t *lrow;             // [rows] first link value of each 64-node row (null with lrec)
  uint32_t vbase;            // elements from the buffer's start to the link values
  uint32_t vcap;             // link values the buffer holds
  int lx, ly, lz;
  int bxn, byn, nbricks, per_xcd;
  Box b;
  const Clock *clk;
  double kax, kdg;  // -6 w_q rho0 of the axis and of the diagonal directions
  H16 h16;
};

// bit q of a mask from a predicate: a 0/1 value shifted into place (no mask constants to keep)
__device__ inline uint32_t pred_bit(bool c, int q) {
  uint32_t b = c ? 1u : 0u;
  asm volatile("" : "+v"(b));
  return b << q;
}
__device__ inline int lane_rank(unsigned long long bl) {  // set bits of bl below this lane
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bl >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bl, 0u));
}

// LDS of a k_links work-group
struct LinksLDS {
  unsigned long long sacc[TS][HYD][2];  // the table's fixed-point sums
  double ssph[TS][9];                    // R, U, W of the table's spheres
  int2 list[LCAP];                       // (table slot, or -1 - sphere; node in the brick | link directions >> 1 << 10)
  int32_t skey[TS];                      // the table's spheres
  uint32_t srec[LBX * LBY * LBZ];        // the brick's link records
  uint32_t srow[LBY * LBZ];              // first link value of each of its rows (k_links: vbase
                                         // included; k_lattice: its index in the brick's slots)
  double spw[4][NPIN];                   // k_lattice: the stream partials of each wave
  int32_t lcount, vcount;
};

// The list and table of one brick; returns the entry count (flags raised go to bad).  The
// records and row starts stay in sh.  FUSED: the row starts index the brick's link slots
// (k_lattice) instead of the link values after the populations.
template <class ST, bool FUSED>
__device__ __forceinline__ int links_list(const LinksArgs &A, int brick, LinksLDS &sh, uint32_t &bad) {
  auto &skey = sh.skey;
  auto &sacc = sh.sacc;
  auto &ssph = sh.ssph;
  auto &list = sh.list;
  auto &lcount = sh.lcount, &vcount = sh.vcount;
  auto &srec = sh.srec;
  auto &srow = sh.srow;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  for (int i = t; i < TS; i += 256) skey[i] = -1;
  for (int i = t; i < TS * HYD * 2; i += 256) (&sacc[0][0][0])[i] = 0ull;
  if (t == 0) { lcount = 0; vcount = 0; }
  __syncthreads();
  const int lx = A.lx, ly = A.ly, lz = A.lz;
  const int x0 = (brick % A.bxn) * LBX, y0 = ((brick / A.bxn) % A.byn) * LBY, z0 = (brick / (A.bxn * A.byn)) * LBZ;
  const int nsl = min(LBZ, lz - z0);
  // ---- list ----
  {
    const __amdgpu_buffer_rsrc_t rown = buf_rsrc(A.own, A.ow_bytes);
    const int x = x0 + lane, y = y0 + wv;
    const bool live = x < lx && y < ly;
    const int xc = live ? x : 0, yc = opaque_uniform(live ? y : y0);
    const int xm = xc == 0 ? lx - 1 : xc - 1, xp = xc + 1 >= lx ? 0 : xc + 1;
    // the lane's byte offsets in a row; the row's goes in the scalar offset (a lane past the
    // box end loads a valid node, whose owner is not used)
    const uint32_t xc4 = (uint32_t)xc * 4u, xm4 = (uint32_t)xm * 4u, xp4 = (uint32_t)xp * 4u;
    int32_t own0[LBZ], so[LBZ][NQ];
#pragma unroll
    for (int sl = 0; sl < LBZ; ++sl) {
      const bool ok = live && sl < nsl;
      const int zo = opaque_uniform(z0 + (sl < nsl ? sl : 0));
      const int32_t o0 = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rown, xc4, (uint32_t)(lx * (yc + ly * zo)) * 4u, 0);
      own0[sl] = ok ? o0 : 0;
      // the nine source rows (y - c_y, z - c_z), wave-uniform; a row next to a sliding plane
      // takes its ghost row there
      const int zu = opaque_uniform(z0 + (sl < nsl ? sl : 0));
      const int zm = zu == 0 ? lz - 1 : zu - 1, zp = zu == lz - 1 ? 0 : zu + 1;
      const int zr[3] = {zp, zu, zm};  // c_z = -1, 0, 1
      int rowb[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) rowb[a][c] = lx * (yc + 1 - a + ly * zr[c]);  // c_y = a - 1
      if (yc == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) rowb[2][c] = A.goff + zr[c] * lx;
      }
      if (yc == ly - 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) rowb[0][c] = A.goff + (lz + zr[c]) * lx;
      }
#pragma unroll
      for (int q = 1; q < NQ; ++q) {
        const uint32_t xs4 = cx(q) == 1 ? xm4 : (cx(q) == -1 ? xp4 : xc4);
        so[sl][q] = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rown, xs4, (uint32_t)rowb[cy(q) + 1][cz(q) + 1] * 4u, 0);
      }
    }
#pragma unroll
    for (int sl = 0; sl < LBZ; ++sl) {
      const bool fl = live && sl < nsl && own0[sl] < 0;
      uint32_t F = 0;       // fluid sources (bit q)
      int32_t smax = -1;    // largest sphere among the sources
      uint32_t smin = ~0u;  // smallest (a fluid source, -1, compares above every sphere)
#pragma unroll
      for (int q = 1; q < NQ; ++q) {
        const int32_t o = so[sl][q];
        F |= ((uint32_t)o >> 31) << q;
        smax = max(smax, o);
        smin = min(smin, (uint32_t)o);
      }
      const uint32_t M = fl ? ~F & 0x7fffeu : 0u;  // link directions
      const bool single = M != 0 && (uint32_t)smax == smin;
      const int loc = lane | (wv << 6) | (sl << 8);
      // the node's record and its row's block of link values
      {
        const int nl = __builtin_popcount(M);
        int pre = 0, tot = 0;
#pragma unroll
        for (int b = 0; b < 5; ++b) {  // exclusive prefix over the wave of nl < 32
          const unsigned long long bl = __ballot((nl >> b) & 1);
          pre += lane_rank(bl) << b;
          tot += __builtin_popcountll(bl) << b;
        }
        const bool ok = live && sl < nsl;
        const uint32_t rec = fl ? (M | ((uint32_t)pre << REC_OFF)) : REC_SOLID;
        int rb = 0;
        if (lane == 0 && ok && tot) rb = atomicAdd(&vcount, tot);
        rb = __builtin_amdgcn_readfirstlane(rb);
        if (rb + tot > LBX * LBY * LBZ * LINK_CAP) bad |= FL_LINKS;  // values past the block are not kept
        const int rl = rb;  // in the brick
        rb += brick * (LBX * LBY * LBZ * LINK_CAP);
        if (!FUSED && ok && A.lrec) {
          const int z = z0 + sl;
          A.lrec[(size_t)xc + (size_t)lx * ((size_t)yc + (size_t)ly * z)] = rec;
          if (lane == 0) A.lrow[(z * ly + yc) * A.bxn + x0 / LBX] = rb;
        }
        srec[loc] = rec;
        if (lane == 0) srow[wv + LBY * sl] = FUSED ? (uint32_t)rl : A.vbase + (uint32_t)rb;
      }
      const unsigned long long bs = __ballot(single);
      int sb = 0;
      if (lane == 0 && bs) sb = atomicAdd(&lcount, __builtin_popcountll(bs));
      sb = __builtin_amdgcn_readfirstlane(sb) + lane_rank(bs);
      if (single && sb < LCAP) list[sb] = make_int2(smax, loc | (int)((M >> 1) << 10));
      if (M != 0 && !single) {  // more than one sphere: in decreasing id
        // the largest first; when the largest of the others is the smallest (two spheres,
        // nearly always) the rest is the second entry, else the others one by one
        uint32_t m1 = 0;
        int32_t s2 = -1;
#pragma unroll
        for (int q = 1; q < NQ; ++q) {
          const bool is1 = so[sl][q] == smax;
          m1 |= pred_bit(is1, q);
          s2 = max(s2, is1 ? -1 : so[sl][q]);
        }
        m1 &= M;
        int pos = atomicAdd(&lcount, 1);
        if (pos < LCAP) list[pos] = make_int2(smax, loc | (int)((m1 >> 1) << 10));
        uint32_t rem = M & ~m1;
        if ((uint32_t)s2 == smin) {
          pos = atomicAdd(&lcount, 1);
          if (pos < LCAP) list[pos] = make_int2(s2, loc | (int)((rem >> 1) << 10));
          rem = 0;
        }
        for (int k = 1; rem != 0; ++k) {
          int32_t sp = -1;
#pragma unroll
          for (int q = 1; q < NQ; ++q) sp = max(sp, ((rem >> q) & 1u) ? so[sl][q] : -1);
          if (k == LMAXS) { bad |= FL_LINKS; break; }
          uint32_t m = 0;
#pragma unroll
          for (int q = 1; q < NQ; ++q) m |= pred_bit(so[sl][q] == sp, q);
          m &= rem;
          rem &= ~m;
          pos = atomicAdd(&lcount, 1);
          if (pos < LCAP) list[pos] = make_int2(sp, loc | (int)((m >> 1) << 10));
        }
      }
    }
  }
  __syncthreads();
  const int cnt0 = lcount;
  if (cnt0 > LCAP) bad |= FL_LINKS;  // links left out: the step reports it
  const int cnt = min(cnt0, LCAP);
  // ---- table: a slot per sphere, the sphere's state staged by the lane that claims it ----
  for (int e = t; e < cnt; e += 256) {
    const int p = list[e].x;
    int h = p & (TS - 1), slot = -1;
    for (int probe = 0; probe < TS; ++probe) {
      int key = skey[h];
      bool mine = false;
      if (key == -1) {
        key = atomicCAS(&skey[h], -1, p);
        mine = key == -1;
      }
      if (mine) {
        for (int c = 0; c < 3; ++c) {
          ssph[h][c] = A.R[3 * p + c];
          ssph[h][3 + c] = A.U[3 * p + c];
          ssph[h][6 + c] = A.W[3 * p + c];
        }
      }
      if (key == -1 || key == p) { slot = h; break; }
      h = (h + 1) & (TS - 1);
    }
    list[e].x = slot >= 0 ? slot : -1 - p;
  }
  __syncthreads();
  return cnt;
}

// The links of one brick (list, table, links, per-sphere sums) for k_stream: each link's
// bounce-back value goes to the link values after the populations.
template <class ST>
__device__ __forceinline__ void links_body(const LinksArgs &A, int brick, LinksLDS &sh) {
  using CT = typename Store<ST>::CT;
  auto &skey = sh.skey;
  auto &sacc = sh.sacc;
  auto &ssph = sh.ssph;
  auto &list = sh.list;
  auto &srec = sh.srec;
  auto &srow = sh.srow;
  uint32_t bad = 0;
  const int cnt = links_list<ST, false>(A, brick, sh, bad);
  const int t = threadIdx.x;
  const int lx = A.lx, ly = A.ly;
  const int x0 = (brick % A.bxn) * LBX, y0 = ((brick / A.bxn) % A.byn) * LBY, z0 = (brick / (A.bxn * A.byn)) * LBZ;
  constexpr uint32_t es = sizeof(ST);
  constexpr uint32_t OOB = 0xfffffff0u;
  // ---- links: one lane per entry; an entry some of whose links end in another image of the
  //      sphere than the one nearest the node is marked and done in a second pass ----
  const Box bx = clock_box(A.b, A.clk, 0);
  const uint32_t pb = (uint32_t)opaque_uniform((int)(A.plane * es));
  const __amdgpu_buffer_rsrc_t rf = buf_rsrc(A.f, A.pop_bytes);
  auto entry = [&](int e, int2 &en, int &key, uint32_t &m, int &x, int &y, int &z) {
    en = list[e];
    key = en.x;
    m = (((uint32_t)en.y >> 10) & 0x3ffffu) << 1;
    x = x0 + (en.y & 63); y = y0 + ((en.y >> 6) & 3); z = z0 + ((en.y >> 8) & 3);
  };
  // the sphere's centre and velocities: staged in LDS, or (a full table) from the arrays
  auto sphere = [&](int key, int c) -> double {
    if (key >= 0) return ssph[key][c];
    const int p = -1 - key;
    return c < 3 ? A.R[3 * p + c] : (c < 6 ? A.U[3 * p + c - 3] : A.W[3 * p + c - 6]);
  };
  // the node's own opposite populations n*_qbar(X) of the links (bounce-back sends them back)
  auto pops = [&](CT (&n)[NQ], uint32_t m, int x, int y, int z) {
    const uint32_t own_base = (uint32_t)(x + lx * (y + ly * z)) * es;
    n[0] = 0;
#pragma unroll
    for (int q = 1; q < NQ; ++q) {
      const uint32_t sel = (uint32_t)__builtin_amdgcn_sbfe((int)m, q, 1);  // all ones on a link
      n[q] = RowIO<ST>::ld(rf, ((opp(q) * pb + own_base) & sel) | (OOB & ~sel), q, A.h16);  // w_qbar = w_q
    }
  };
  // element of the link value of direction q of the node at loc (q must be a link of it)
  // (the node's record and the element of its first value, read once per entry: vfirst)
  auto vfirst = [&](int loc, uint32_t &rec) -> uint32_t {
    rec = srec[loc];
    const uint32_t e = srow[(loc >> 6) & 15] + (rec >> REC_OFF);
    // a node whose values pass the brick's block (reported with FL_LINKS): the array's end,
    // where nothing is written
    return e + __builtin_popcount(rec) <= A.vbase + (uint32_t)(brick + 1) * (LBX * LBY * LBZ * LINK_CAP)
               ? e : A.vbase + A.vcap;
  };
  auto vslot = [&](uint32_t v0, uint32_t rec, int q) -> uint32_t {
    return v0 + __builtin_popcount(rec & ((1u << q) - 2u));
  };
  // the entry's sums into the table (a full table: straight into the sphere's sums)
  auto add = [&](int key, uint32_t m, const double (&v)[HYD]) {
    if (key >= 0) {
#pragma unroll
      for (int c = 0; c < HYD - 1; ++c) fx_lds(as_lds(&sacc[key][c][0]), v[c]);
      __hip_atomic_fetch_add(as_lds(&sacc[key][HYD - 1][0]), (unsigned long long)__builtin_popcount(m) << FXH,
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);  // an integer
    } else {
      unsigned long long *d = &A.hacc[(size_t)(-1 - key) * HYD * 2];
      for (int c = 0; c < HYD - 1; ++c) fx_add(d + 2 * c, v[c]);
      atomicAdd(d + 2 * (HYD - 1), (unsigned long long)__builtin_popcount(m) << FXH);
    }
  };
  const double ilx = 1.0 / bx.Lx, ilz = 1.0 / bx.Lz;
  for (int e = t; e < cnt; e += 256) {
    int2 en;
    int key, x, y, z;
    uint32_t m;
    entry(e, en, key, m, x, y, z);
    CT n[NQ];
    pops(n, m, x, y, z);
    double Dx, Dy, Dz;
    int k;
    node_image(bx, ilx, ilz, (double)x - sphere(key, 0), (double)y - sphere(key, 1), (double)z - sphere(key, 2),
               Dx, Dy, Dz, k);
    if (!links_in_image(m, bx, Dx, Dy, Dz)) {  // some link ends in another image
      list[e].y = en.y | (int)0x80000000;
      continue;
    }
    const double w0 = sphere(key, 6), w1 = sphere(key, 7), w2 = sphere(key, 8);
    // rigid-body velocity at the node (eq. 8)
    const double ux = sphere(key, 3) + k * bx.ule + (w1 * Dz - w2 * Dy);
    const double uy = sphere(key, 4) + (w2 * Dx - w0 * Dz);
    const double uz = sphere(key, 5) + (w0 * Dy - w1 * Dx);
    uint32_t rec;
    const uint32_t v0 = vfirst(en.y & 1023, rec);
    double g0 = 0, g1 = 0, g2 = 0, mxx = 0, myy = 0, mzz = 0, mxy = 0, mxz = 0, myz = 0;
#pragma unroll
    for (int pi = 0; pi < 9; ++pi) {
      const int q = 2 * pi + 1, b = q + 1;
      const double corr = (q <= 6 ? A.kax : A.kdg) * cdot<double>(q, ux, uy, uz);
      const bool lq = (m >> q) & 1u, lb = (m >> b) & 1u;
      const double mq = lq ? fma(2.0, (double)n[q], -corr) : 0.0;
      const double mb = lb ? fma(2.0, (double)n[b], corr) : 0.0;
      const double sm2 = mq + mb, df = mq - mb;
      // each sum starts at its first contributing pair (no addition to zero)
      acc_pair(g0, pi, 0, cx(q), df); acc_pair(g1, pi, 1, cy(q), df); acc_pair(g2, pi, 2, cz(q), df);
      acc_pair(mxx, pi, 0, cx(q) * cx(q), sm2);
      acc_pair(myy, pi, 1, cy(q) * cy(q), sm2);
      acc_pair(mzz, pi, 2, cz(q) * cz(q), sm2);
      acc_pair(mxy, pi, 3, cx(q) * cy(q), sm2); acc_pair(mxz, pi, 4, cx(q) * cz(q), sm2);
      acc_pair(myz, pi, 5, cy(q) * cz(q), sm2);
      // the bounce-back values into the link values
      RowIO<ST>::st(rf, lq ? vslot(v0, rec, q) * es : OOB, (CT)((double)n[q] - corr), q, A.h16);
      RowIO<ST>::st(rf, lb ? vslot(v0, rec, b) * es : OOB, (CT)((double)n[b] + corr), b, A.h16);
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
    v[12] = 0.0;  // the link count is added from m
    add(key, m, v);
  }
  // the marked entries: each link with the lever and velocity of the image holding its solid
  // end (eq. 8); the lever of link q is its midpoint X - c_q/2 minus that image's centre
  for (int e = t; e < cnt; e += 256) {
    if (list[e].y >= 0) continue;
    int2 en;
    int key, x, y, z;
    uint32_t m;
    entry(e, en, key, m, x, y, z);
    const int p = key >= 0 ? skey[key] : -1 - key;  // the sphere's state from its arrays here
    const uint32_t own_base = (uint32_t)(x + lx * (y + ly * z)) * es;
    double v[HYD];
#pragma unroll
    for (int c = 0; c < HYD; ++c) v[c] = 0.0;
#pragma unroll 1
    for (int q = 1; q < NQ; ++q) {  // not unrolled: a rare path, kept small
      if (!((m >> q) & 1u)) continue;
      const int qx = cx(q), qy = cy(q), qz = cz(q);
      double ex, ey, ez;
      int kq;
      minimage(bx, (double)(x - qx) - A.R[3 * p], (double)(y - qy) - A.R[3 * p + 1],
               (double)(z - qz) - A.R[3 * p + 2], ex, ey, ez, kq);
      const double lvx = ex + 0.5 * qx, lvy = ey + 0.5 * qy, lvz = ez + 0.5 * qz;
      const double w0 = A.W[3 * p], w1 = A.W[3 * p + 1], w2 = A.W[3 * p + 2];
      const double ubx = A.U[3 * p] + kq * bx.ule + (w1 * lvz - w2 * lvy);
      const double uby = A.U[3 * p + 1] + (w2 * lvx - w0 * lvz);
      const double ubz = A.U[3 * p + 2] + (w0 * lvy - w1 * lvx);
      double cu = 0.0;  // c_q . u_b, x y z in order
      bool first = true;
      if (qx != 0) { cu = qx > 0 ? ubx : -ubx; first = false; }
      if (qy != 0) { const double t1 = qy > 0 ? uby : -uby; cu = first ? t1 : cu + t1; first = false; }
      if (qz != 0) { const double t1 = qz > 0 ? ubz : -ubz; cu = first ? t1 : cu + t1; }
      const double corr = (q <= 6 ? A.kax : A.kdg) * cu;
      const double fo = (double)RowIO<ST>::ld(rf, opp(q) * pb + own_base, q, A.h16);
      uint32_t rec;
      const uint32_t v0 = vfirst(en.y & 1023, rec);
      RowIO<ST>::st(rf, vslot(v0, rec, q) * es, (CT)(fo - corr), q, A.h16);
      const double mm = fma(2.0, fo, -corr);
      double f[3] = {0.0, 0.0, 0.0};
      addc(f[0], -qx, mm); addc(f[1], -qy, mm); addc(f[2], -qz, mm);
      v[0] += f[0]; v[1] += f[1]; v[2] += f[2];
      v[3] += lvy * f[2] - lvz * f[1];
      v[4] += lvz * f[0] - lvx * f[2];
      v[5] += lvx * f[1] - lvy * f[0];
      v[6] += lvx * f[0]; v[7] += lvy * f[1]; v[8] += lvz * f[2];
      v[9] += 0.5 * (lvx * f[1] + lvy * f[0]);
      v[10] += 0.5 * (lvx * f[2] + lvz * f[0]);
      v[11] += 0.5 * (lvy * f[2] + lvz * f[1]);
    }
    add(key, m, v);
  }
  if (bad) atomicOr(A.flags, (int32_t)bad);
  __syncthreads();
  for (int i = t; i < TS * HYD; i += 256) {
    const int slot = i / HYD, c = i - slot * HYD;
    const int key = skey[slot];
    if (key >= 0) {
      const unsigned long long h = sacc[slot][c][0], l = sacc[slot][c][1];
      if (h | l) {
        atomicAdd(&A.hacc[((size_t)key * HYD + c) * 2], h);
        atomicAdd(&A.hacc[((size_t)key * HYD + c) * 2 + 1], l);
      }
    }
  }
}

// ---- k_lattice's link phases.  Its stream phase takes a link's own opposite population
// n*_qbar(X) from the populations itself (those lines are in the L2 for the brick's own pulls)
// and the link's correction from the brick's link slots, where it leaves n*_qbar(X) for the
// sums; so no phase reads the populations twice, and the slots live in LDS:
//   pre   one lane per entry: corr = -6 w_q rho0 u(X) . c_q of each link into its slot
//   sums  one lane per entry, m = 2 n*_qbar - corr and the entry's F, T, S as in k_links; the
//         entries are taken in a scattered order, so that the lanes of a wave meet at fewer
//         spheres in the table's atomics
// Slot k of a brick (k < LINK_CAP values per node): LDS for k < VLDS, else the brick's block
// of link values after the populations, read as the compute type (a brick with more links
// than VLDS; the 256^3 bulk suspension at phi 0.55 has 1,573 per brick on average, 2,564 at
// most).  Bricks within VLDS (OVF false) run without branches: a direction that is no link
// of the lane's node takes the lane's spare slot VLDS + lane, which always holds 0.
constexpr int VLDS = 2560;
constexpr int BRICK_VALUES = LBX * LBY * LBZ * LINK_CAP;
template <class CT> struct CtIO;
template <> struct CtIO<float> {
  __device__ static float ld(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  }
  __device__ static void st(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 0);
  }
};
template <> struct CtIO<double> {
  __device__ static double ld(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  }
  __device__ static void st(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
  }
};
template <class CT> struct LinkSlots {
  CT *lds;
  __amdgpu_buffer_rsrc_t r;  // the population buffer
  uint32_t block;            // byte offset of the brick's block of link values
  bool ovf;                  // more than VLDS links in the brick (work-group uniform)
  __device__ uint32_t goff(uint32_t k) const {  // past the block: nothing kept (FL_LINKS raised)
    return k < (uint32_t)BRICK_VALUES ? block + (k - VLDS) * (uint32_t)sizeof(CT) : 0xfffffff0u;
  }
  __device__ CT ld(uint32_t k) const {
    if (!ovf) return lds[k];
    return k < (uint32_t)VLDS ? lds[k] : CtIO<CT>::ld(r, goff(k));
  }
  __device__ void st(uint32_t k, CT v) const {
    if (!ovf) { lds[k] = v; return; }
    if (k < (uint32_t)VLDS) lds[k] = v;
    else CtIO<CT>::st(r, goff(k), v);
  }
};

// centre, velocity and spin of an entry's sphere: staged in the table, or (a full table) from
// the arrays
__device__ inline double sph_state(const LinksArgs &A, const LinksLDS &sh, int key, int c) {
  if (key >= 0) return sh.ssph[key][c];
  const int p = -1 - key;
  return c < 3 ? A.R[3 * p + c] : (c < 6 ? A.U[3 * p + c - 3] : A.W[3 * p + c - 6]);
}
// The node's lever D (node minus the nearest image of the centre) and the rigid-body velocity
// there (eq. 8); false when some link of m ends in another image (the per-link path).
__device__ inline bool entry_motion(const LinksArgs &A, const LinksLDS &sh, const Box &bx, int key, uint32_t m,
                                    int x, int y, int z, double &Dx, double &Dy, double &Dz, double &ux, double &uy,
                                    double &uz) {
  const double ilx = 1.0 / bx.Lx, ilz = 1.0 / bx.Lz;
  int k;
  node_image(bx, ilx, ilz, (double)x - sph_state(A, sh, key, 0), (double)y - sph_state(A, sh, key, 1),
             (double)z - sph_state(A, sh, key, 2), Dx, Dy, Dz, k);
  if (!links_in_image(m, bx, Dx, Dy, Dz)) return false;
  const double w0 = sph_state(A, sh, key, 6), w1 = sph_state(A, sh, key, 7), w2 = sph_state(A, sh, key, 8);
  ux = sph_state(A, sh, key, 3) + k * bx.ule + (w1 * Dz - w2 * Dy);
  uy = sph_state(A, sh, key, 4) + (w2 * Dx - w0 * Dz);
  uz = sph_state(A, sh, key, 5) + (w0 * Dy - w1 * Dx);
  return true;
}
// Per-link path: the lever of link q (its midpoint X - c_q/2 minus the centre of the image
// holding its solid end) and its correction -6 w_q rho0 u_b . c_q.
__device__ inline double link_corr(const LinksArgs &A, const Box &bx, int p, int x, int y, int z, int q,
                                   double &lvx, double &lvy, double &lvz) {
  const int qx = cx(q), qy = cy(q), qz = cz(q);
  double ex, ey, ez;
  int kq;
  minimage(bx, (double)(x - qx) - A.R[3 * p], (double)(y - qy) - A.R[3 * p + 1], (double)(z - qz) - A.R[3 * p + 2],
           ex, ey, ez, kq);
  lvx = ex + 0.5 * qx; lvy = ey + 0.5 * qy; lvz = ez + 0.5 * qz;
  const double w0 = A.W[3 * p], w1 = A.W[3 * p + 1], w2 = A.W[3 * p + 2];
  const double ubx = A.U[3 * p] + kq * bx.ule + (w1 * lvz - w2 * lvy);
  const double uby = A.U[3 * p + 1] + (w2 * lvx - w0 * lvz);
  const double ubz = A.U[3 * p + 2] + (w0 * lvy - w1 * lvx);
  double cu = 0.0;  // c_q . u_b, x y z in order
  bool first = true;
  if (qx != 0) { cu = qx > 0 ? ubx : -ubx; first = false; }
  if (qy != 0) { const double t1 = qy > 0 ? uby : -uby; cu = first ? t1 : cu + t1; first = false; }
  if (qz != 0) { const double t1 = qz > 0 ? ubz : -ubz; cu = first ? t1 : cu + t1; }
  return (q <= 6 ? A.kax : A.kdg) * cu;
}
// An entry's sums into the table (a full table: straight into the sphere's sums).
__device__ inline void table_add(const LinksArgs &A, LinksLDS &sh, int key, uint32_t m, const double (&v)[HYD]) {
  if (key >= 0) {
#pragma unroll
    for (int c = 0; c < HYD - 1; ++c) fx_lds(as_lds(&sh.sacc[key][c][0]), v[c]);
    __hip_atomic_fetch_add(as_lds(&sh.sacc[key][HYD - 1][0]), (unsigned long long)__builtin_popcount(m) << FXH,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);  // an integer
  } else {
    unsigned long long *d = &A.hacc[(size_t)(-1 - key) * HYD * 2];
    for (int c = 0; c < HYD - 1; ++c) fx_add(d + 2 * c, v[c]);
    atomicAdd(d + 2 * (HYD - 1), (unsigned long long)__builtin_popcount(m) << FXH);
  }
}
// the table's sums into the spheres' sums
__device__ inline void table_flush(const LinksArgs &A, const LinksLDS &sh) {
  for (int i = threadIdx.x; i < TS * HYD; i += 256) {
    const int slot = i / HYD, c = i - slot * HYD;
    const int key = sh.skey[slot];
    if (key >= 0) {
      const unsigned long long h = sh.sacc[slot][c][0], l = sh.sacc[slot][c][1];
      if (h | l) {
        atomicAdd(&A.hacc[((size_t)key * HYD + c) * 2], h);
        atomicAdd(&A.hacc[((size_t)key * HYD + c) * 2 + 1], l);
      }
    }
  }
}
// slot of link q of a node whose first slot is v0 (q a link of the record)
__device__ inline uint32_t rec_slot(uint32_t v0, uint32_t rec, int q) {
  return v0 + __builtin_popcount(rec & ((1u << q) - 2u));
}

// pre: the corrections of the brick's links into their slots; entries whose links may end in
// another image are marked and done per link.
template <class ST, bool OVF>
__device__ __forceinline__ void lattice_pre(const LinksArgs &A, int brick, LinksLDS &sh,
                                            const LinkSlots<typename Store<ST>::CT> &S, int cnt) {
  using CT = typename Store<ST>::CT;
  const int t = threadIdx.x;
  const uint32_t spare = VLDS + (t & 63);
  const int x0 = (brick % A.bxn) * LBX, y0 = ((brick / A.bxn) % A.byn) * LBY, z0 = (brick / (A.bxn * A.byn)) * LBZ;
  const Box bx = clock_box(A.b, A.clk, 0);
  for (int e = t; e < cnt; e += 256) {
    const int2 en = sh.list[e];
    const int key = en.x, loc = en.y & 1023;
    const uint32_t m = (((uint32_t)en.y >> 10) & 0x3ffffu) << 1;
    const int x = x0 + (loc & 63), y = y0 + ((loc >> 6) & 3), z = z0 + ((loc >> 8) & 3);
    double Dx, Dy, Dz, ux, uy, uz;
    if (!entry_motion(A, sh, bx, key, m, x, y, z, Dx, Dy, Dz, ux, uy, uz)) {
      sh.list[e].y = en.y | (int)0x80000000;
      continue;
    }
    const uint32_t rec = sh.srec[loc];
    uint32_t kn = sh.srow[(loc >> 6) & 15] + (rec >> REC_OFF);  // the slot of the node's next link
#pragma unroll
    for (int pi = 0; pi < 9; ++pi) {
      const int q = 2 * pi + 1, b = q + 1;
      const double corr = (q <= 6 ? A.kax : A.kdg) * cdot<double>(q, ux, uy, uz);
      const bool lq = (m >> q) & 1u, lb = (m >> b) & 1u;
      const uint32_t kq = kn;
      kn += (rec >> q) & 1u;
      const uint32_t kb = kn;
      kn += (rec >> b) & 1u;
      if constexpr (OVF) {
        if (lq) S.st(kq, (CT)corr);
        if (lb) S.st(kb, (CT)(-corr));  // c_b = -c_q
      } else {
        S.lds[lq ? kq : spare] = lq ? (CT)corr : (CT)0;
        S.lds[lb ? kb : spare] = lb ? (CT)(-corr) : (CT)0;
      }
    }
  }
  for (int e = t; e < cnt; e += 256) {  // the marked entries (this thread's own)
    const int2 en = sh.list[e];
    if (en.y >= 0) continue;
    const int key = en.x, loc = en.y & 1023;
    const uint32_t m = (((uint32_t)en.y >> 10) & 0x3ffffu) << 1;
    const int x = x0 + (loc & 63), y = y0 + ((loc >> 6) & 3), z = z0 + ((loc >> 8) & 3);
    const int p = key >= 0 ? sh.skey[key] : -1 - key;
    const uint32_t rec = sh.srec[loc];
    const uint32_t v0 = sh.srow[(loc >> 6) & 15] + (rec >> REC_OFF);
#pragma unroll 1
    for (int q = 1; q < NQ; ++q) {  // a rare path, kept small
      if (!((m >> q) & 1u)) continue;
      double lvx, lvy, lvz;
      S.st(rec_slot(v0, rec, q), (CT)link_corr(A, bx, p, x, y, z, q, lvx, lvy, lvz));
    }
  }
}

// sums: the exchanged momentum of every link from n*_qbar(X) left in its slot by the stream
// phase, summed per entry (F = -sum m c_q, T = D x F, S = sym(D (x) F) + 1/2 sum m c_q c_q) into
// the table, then into the spheres' sums.
template <class ST, bool OVF>
__device__ __forceinline__ void lattice_sums(const LinksArgs &A, int brick, LinksLDS &sh,
                                             const LinkSlots<typename Store<ST>::CT> &S, int cnt, uint32_t bad) {
  const int t = threadIdx.x;
  const int x0 = (brick % A.bxn) * LBX, y0 = ((brick / A.bxn) % A.byn) * LBY, z0 = (brick / (A.bxn * A.byn)) * LBZ;
  const Box bx = clock_box(A.b, A.clk, 0);
  // entry (j P) mod cnt for j = t, t + 256, ...: a permutation (P prime, not a divisor of cnt)
  const int P = cnt % 97 ? 97 : 89;
  const int cn = cnt > 0 ? cnt : 1;
  const int stride = (256 * P) % cn;
  int e = (t * P) % cn;
  for (int j = t; j < cnt; j += 256) {
    const int2 en = sh.list[e];
    e += stride;
    e -= e >= cnt ? cnt : 0;
    if (en.y < 0) continue;  // marked: below
    const int key = en.x, loc = en.y & 1023;
    const uint32_t m = (((uint32_t)en.y >> 10) & 0x3ffffu) << 1;
    const int x = x0 + (loc & 63), y = y0 + ((loc >> 6) & 3), z = z0 + ((loc >> 8) & 3);
    double Dx, Dy, Dz, ux, uy, uz;
    entry_motion(A, sh, bx, key, m, x, y, z, Dx, Dy, Dz, ux, uy, uz);  // true: not marked
    const uint32_t rec = sh.srec[loc];
    const uint32_t v0 = sh.srow[(loc >> 6) & 15] + (rec >> REC_OFF);
    // the slot of the node's next link direction (a running count over the record's bits);
    // a direction that is no link of the entry reads some slot within the array, unused
    uint32_t kn = v0;
    double g0 = 0, g1 = 0, g2 = 0, mxx = 0, myy = 0, mzz = 0, mxy = 0, mxz = 0, myz = 0;
#pragma unroll
    for (int pi = 0; pi < 9; ++pi) {
      const int q = 2 * pi + 1, b = q + 1;
      const double corr = (q <= 6 ? A.kax : A.kdg) * cdot<double>(q, ux, uy, uz);
      const bool lq = (m >> q) & 1u, lb = (m >> b) & 1u;
      const uint32_t kq = kn;
      kn += (rec >> q) & 1u;
      const uint32_t kb = kn;
      kn += (rec >> b) & 1u;
      double nq, nb;  // n*_qbar(X), n*_bbar(X)
      if constexpr (OVF) {
        nq = lq ? (double)S.ld(kq) : 0.0;
        nb = lb ? (double)S.ld(kb) : 0.0;
      } else {
        nq = (double)S.lds[kq];
        nb = (double)S.lds[kb];
      }
      const double mq = lq ? fma(2.0, nq, -corr) : 0.0;
      const double mb = lb ? fma(2.0, nb, corr) : 0.0;
      const double sm2 = mq + mb, df = mq - mb;
      // each sum starts at its first contributing pair (no addition to zero)
      acc_pair(g0, pi, 0, cx(q), df); acc_pair(g1, pi, 1, cy(q), df); acc_pair(g2, pi, 2, cz(q), df);
      acc_pair(mxx, pi, 0, cx(q) * cx(q), sm2);
      acc_pair(myy, pi, 1, cy(q) * cy(q), sm2);
      acc_pair(mzz, pi, 2, cz(q) * cz(q), sm2);
      acc_pair(mxy, pi, 3, cx(q) * cy(q), sm2); acc_pair(mxz, pi, 4, cx(q) * cz(q), sm2);
      acc_pair(myz, pi, 5, cy(q) * cz(q), sm2);
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
    v[12] = 0.0;  // the link count is added from m
    table_add(A, sh, key, m, v);
  }
  for (int e2 = t; e2 < cnt; e2 += 256) {  // the marked entries: each link with its own lever
    const int2 en = sh.list[e2];
    if (en.y >= 0) continue;
    const int key = en.x, loc = en.y & 1023;
    const uint32_t m = (((uint32_t)en.y >> 10) & 0x3ffffu) << 1;
    const int x = x0 + (loc & 63), y = y0 + ((loc >> 6) & 3), z = z0 + ((loc >> 8) & 3);
    const int p = key >= 0 ? sh.skey[key] : -1 - key;
    const uint32_t rec = sh.srec[loc];
    const uint32_t v0 = sh.srow[(loc >> 6) & 15] + (rec >> REC_OFF);
    double v[HYD];
#pragma unroll
    for (int c = 0; c < HYD; ++c) v[c] = 0.0;
#pragma unroll 1
    for (int q = 1; q < NQ; ++q) {
      if (!((m >> q) & 1u)) continue;
      double lvx, lvy, lvz;
      const double corr = link_corr(A, bx, p, x, y, z, q, lvx, lvy, lvz);
      const double mm = fma(2.0, (double)S.ld(rec_slot(v0, rec, q)), -corr);
      double f[3] = {0.0, 0.0, 0.0};
      addc(f[0], -cx(q), mm); addc(f[1], -cy(q), mm); addc(f[2], -cz(q), mm);
      v[0] += f[0]; v[1] += f[1]; v[2] += f[2];
      v[3] += lvy * f[2] - lvz * f[1];
      v[4] += lvz * f[0] - lvx * f[2];
      v[5] += lvx * f[1] - lvy * f[0];
      v[6] += lvx * f[0]; v[7] += lvy * f[1]; v[8] += lvz * f[2];
      v[9] += 0.5 * (lvx * f[1] + lvy * f[0]);
      v[10] += 0.5 * (lvx * f[2] + lvz * f[0]);
      v[11] += 0.5 * (lvy * f[2] + lvz * f[1]);
    }
    table_add(A, sh, key, m, v);
  }
  if (bad) atomicOr(A.flags, (int32_t)bad);
  __syncthreads();
  table_flush(A, sh);
}

template <class ST>
__global__ __launch_bounds__(256) void k_links(LinksArgs A) {
  __shared__ LinksLDS sh;
  const int brick = (blockIdx.x & 7) * A.per_xcd + (blockIdx.x >> 3);
  if (brick >= A.nbricks) return;  // the whole work-group
  links_body<ST>(A, brick, sh);
}

// ---- k_stream ----
// A brick of 64 x BY x BZ nodes per work-group, dealt to the 8 XCDs in contiguous ranges so
// that neighbouring bricks share an L2.  Wave w takes rows y_lo + w, y_lo + w + 4, ... and
// walks each through the brick's z range (the owner word of the next node loaded a step
// ahead); the waves never wait for each other.  The brick's partials of the fluid stress
// and mass are summed in a fixed order.
// COLL 0: BGK; 1: the linearised operator with separate eigenvalues for the traceless
// stress (-1/tau), its trace (-1/tau_bulk) and the ghost modes (-1/tau_ghost).
struct StreamArgs {
  const void *fin;
  void *fout;
  size_t plane;
  uint32_t pop_bytes, gval_bytes, rec_bytes;
  const uint32_t *lrec;  // link records of the step (k_links)
  const int32_t *lrow;   // first link value of each 64-node row
  uint32_t vbase;        // elements from a population buffer's start to its link values
  const void *gval;
  double *pin;  // [nbricks][NPIN]
  int32_t *flags;
  int lx, ly, lz;
  int bxn, byn, BY, BZ, nbricks, per_xcd;
  double rho0, omega;
  double om_ghost, om_bulk;  // multi-eigenvalue collision: -lambda_g, -lambda_v
  H16 h16;
};

// The end of a brick's stream phase: its lanes' flags and health counters, and the brick's
// partials of the fluid stress and mass (the 256 per-thread partials of each component summed by
// one wave in a fixed order; spn is LDS of the work-group).
template <class CT>
__device__ __forceinline__ void stream_tail(const StreamArgs &A, int brick, CT (*spn)[256], const CT (&pacc)[NPIN],
                                            uint32_t bad, uint32_t nfast, CT umax) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  if (bad) atomicOr(A.flags, (int32_t)bad);  // rare
  if (nfast) {  // rare: the health counters (count of fast node-steps, largest u^2 as bits)
    atomicAdd((unsigned long long *)(A.flags + FL_HEALTH), (unsigned long long)nfast);
    atomicMax(A.flags + FL_HEALTH + 2, __float_as_int((float)umax));
  }
#pragma unroll
  for (int c = 0; c < NPIN; ++c) spn[c][t] = pacc[c];
  __syncthreads();
  if (wv == 0) {
#pragma unroll
    for (int c = 0; c < NPIN; ++c) {
      const double v = wave_sum(((double)spn[c][lane] + (double)spn[c][lane + 64]) +
                                ((double)spn[c][lane + 128] + (double)spn[c][lane + 192]));
      if (lane == 0) A.pin[(size_t)brick * NPIN + c] = v;
    }
  }
}

// One node of the stream phase: pull (eq. 3), collision (eqs. 4, 5) on the deviations, the
// node's partials, and its row store (every lane of a row stores, solid nodes as the rest
// state, never read, so that the wave writes whole cache lines: HBM3E has no write mask, and a
// partly written line costs a read-modify-write).  rec: the node's link record (REC_SOLID for a
// lane past the box end); vrow: its row's first link value.  A link takes its bounce-back value
// n*_qbar(X) - corr (eq. 7): k_stream reads it whole from the link values (k_links wrote it);
// in k_lattice (FUSED) the node loads its own n*_qbar(X), takes corr from the link's slot and
// leaves n*_qbar(X) there for the sums.
template <class ST, int COLL, int FUSED>  // FUSED 0: k_stream; 1, 2: k_lattice (2: slots past VLDS)
__device__ __forceinline__ void stream_node(const StreamArgs &A, __amdgpu_buffer_rsrc_t rin,
                                            __amdgpu_buffer_rsrc_t rout, __amdgpu_buffer_rsrc_t rgh, uint32_t pb,
                                            int x, int y, int z, bool xin, uint32_t rec, uint32_t vrow,
                                            typename Store<ST>::CT (&pacc)[NPIN], uint32_t &bad, uint32_t &nfast,
                                            typename Store<ST>::CT &umax,
                                            const LinkSlots<typename Store<ST>::CT> &S) {
  using CT = typename Store<ST>::CT;
  constexpr uint32_t es = sizeof(ST), ges = sizeof(CT);
  const int lx = A.lx, ly = A.ly, lz = A.lz;
  const CT om = (CT)A.omega;
  const CT rho0 = (CT)A.rho0;
  const uint32_t rowc = (uint32_t)((z * ly + y) * lx) * es;  // byte offset of the row in a plane
  CT n[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) n[q] = 0;  // a solid node stores the rest state
  if (!(rec & REC_SOLID)) {  // fluid node (a lane past the box end reads as solid)
  const int xm = x == 0 ? lx - 1 : x - 1, xp = x + 1 >= lx ? 0 : x + 1;
  const uint32_t xcb = x * es, xmb = xm * es, xpb = xp * es;
  const uint32_t xcg = x * ges, xmg = xm * ges, xpg = xp * ges;
  const int zm = z == 0 ? lz - 1 : z - 1, zp = z == lz - 1 ? 0 : z + 1;
  // ---- pull (eq. 3); a link takes its bounce-back value from the link values (k_links),
  //      the node's own after each other in direction order ----
  const uint32_t v0 = vrow + (rec >> REC_OFF);
  n[0] = RowIO<ST>::ld(rin, rowc + xcb, 0, A.h16);
#pragma unroll
  for (int q = 1; q < NQ; ++q) {
    const int ys = y - cy(q);
    const int zs = cz(q) == 1 ? zm : (cz(q) == -1 ? zp : z);
    const uint32_t xsb = cx(q) == 1 ? xmb : (cx(q) == -1 ? xpb : xcb);
    // across a sliding plane this reads some other row, or nothing; replaced below
    const uint32_t pull = q * pb + (uint32_t)((zs * ly + ys) * lx) * es + xsb;
    const uint32_t link = FUSED ? opp(q) * pb + rowc + xcb  // n*_qbar at the node itself
                                : (v0 + __builtin_popcount(rec & ((1u << q) - 2u))) * es;
    n[q] = RowIO<ST>::ld(rin, ((rec >> q) & 1u) ? link : pull, q, A.h16);
  }
  if (y == 0 || y == ly - 1) {  // directions across the sliding plane: the ghost row
    const int side = y == 0 ? 0 : 1;
#pragma unroll
    for (int q = 1; q < NQ; ++q) {
      if (cy(q) == (side == 0 ? 1 : -1)) {
        const int zs = cz(q) == 1 ? zm : (cz(q) == -1 ? zp : z);
        const uint32_t xsg = cx(q) == 1 ? xmg : (cx(q) == -1 ? xpg : xcg);
        if (!((rec >> q) & 1u))  // a link keeps its bounce-back value
          n[q] = RowIO<CT>::ld(rgh, (uint32_t)(((side * 5 + gslot(q)) * lz + zs) * lx) * ges + xsg, q, A.h16);
      }
    }
  }
  if constexpr (FUSED == 1) {  // the corrections out of the slots, n*_qbar(X) in (one exchange)
    const uint32_t spare = VLDS + (threadIdx.x & 63);
    uint32_t kn = v0;  // the slot of the node's next link direction
#pragma unroll
    for (int q = 1; q < NQ; ++q) {
      const bool lk = (rec >> q) & 1u;
      CT *const slot = S.lds + (lk ? kn : spare);
      kn += lk ? 1u : 0u;
      n[q] -= __hip_atomic_exchange(slot, lk ? n[q] : (CT)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  } else if constexpr (FUSED == 2) {
#pragma unroll
    for (int q = 1; q < NQ; ++q) {
      if ((rec >> q) & 1u) {
        const uint32_t k = rec_slot(v0, rec, q);
        const CT c = S.ld(k);
        S.st(k, n[q]);
        n[q] -= c;
      }
    }
  }
  // ---- moments and collision on the deviations d_q = n_q - w_q rho0, opposite
  //      directions paired: feq_q,qbar = w (a + 4.5 rho cu^2) +- 3 w rho cu ----
  CT rd = n[0], jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int pi = 0; pi < 9; ++pi) {
    const int q = 2 * pi + 1;
    const CT dq = n[q] - n[q + 1];
    rd += n[q] + n[q + 1];
    addc(jx, cx(q), dq); addc(jy, cy(q), dq); addc(jz, cz(q), dq);
  }
  const CT rho = rho0 + rd;
  const CT ir = recip(rho);
  const CT ux = jx * ir, uy = jy * ir, uz = jz * ir;
  const CT uu = ux * ux + uy * uy + uz * uz;
  // a non-finite density or velocity: the fluid has failed.  Speeds above 0.3 c_s (u^2 >
  // 0.03, past the low-Mach range) are counted, not failed: a node squeezed into a one-node
  // gap between two surfaces passes it briefly in dense runs
  bad |= isfinite(uu) && isfinite(rho) ? 0u : (uint32_t)FL_FLUID;
  nfast += uu > (CT)0.03 ? 1u : 0u;
  umax = uu > umax ? uu : umax;
  const CT a = rd - (CT)1.5 * rho * uu;
  const CT w0 = (CT)(1.0 / 3.0), w1 = (CT)(1.0 / 18.0), w2 = (CT)(1.0 / 36.0);
  const CT a1 = w1 * a, a2 = w2 * a;
  const CT b1 = (CT)4.5 * w1 * rho, b2 = (CT)4.5 * w2 * rho;
  const CT c1 = (CT)3 * w1 * rho, c2 = (CT)3 * w2 * rho;
  CT ps[9];
  if constexpr (COLL == 0) {
    n[0] = fmaT(-om, n[0] - w0 * a, n[0]);
#pragma unroll
    for (int pi = 0; pi < 9; ++pi) {
      const int q = 2 * pi + 1, b = q + 1;
      const CT cu = cdot<CT>(q, ux, uy, uz);
      const CT sym = fmaT(q <= 6 ? b1 : b2, cu * cu, q <= 6 ? a1 : a2);
      const CT anti = (q <= 6 ? c1 : c2) * cu;
      const CT neq = n[q] - (sym + anti), neb = n[b] - (sym - anti);
      ps[pi] = neq + neb;
      n[q] = fmaT(-om, neq, n[q]);
      n[b] = fmaT(-om, neb, n[b]);
    }
  } else {
    // n* = n^eq + (1 - om_g) n^neq + Q_q, Q_q = 4.5 w_q [g1 (Pi:c c - t/3) + g2 t (|c|^2 - 1)/3]
    // with Pi = Pi^neq, t its trace, g1 = om_g - om, g2 = om - om_v: the traceless
    // stress relaxes with om, its trace with om_v, every other mode with om_g
    const CT omg = (CT)A.om_ghost, g1 = omg - om, g2 = om - (CT)A.om_bulk;
    const CT ne0 = n[0] - w0 * a;
#pragma unroll
    for (int pi = 0; pi < 9; ++pi) {  // n^neq into n, pair sums for the flux
      const int q = 2 * pi + 1, b = q + 1;
      const CT cu = cdot<CT>(q, ux, uy, uz);
      const CT sym = fmaT(q <= 6 ? b1 : b2, cu * cu, q <= 6 ? a1 : a2);
      const CT anti = (q <= 6 ? c1 : c2) * cu;
      n[q] = n[q] - (sym + anti);
      n[b] = n[b] - (sym - anti);
      ps[pi] = n[q] + n[b];
    }
    CT P[6] = {0, 0, 0, 0, 0, 0};  // xx yy zz xy xz yz
#pragma unroll
    for (int pi = 0; pi < 9; ++pi) {
      const int q = 2 * pi + 1;
      if (cx(q) != 0) P[0] += ps[pi];
      if (cy(q) != 0) P[1] += ps[pi];
      if (cz(q) != 0) P[2] += ps[pi];
      addc(P[3], cx(q) * cy(q), ps[pi]);
      addc(P[4], cx(q) * cz(q), ps[pi]);
      addc(P[5], cy(q) * cz(q), ps[pi]);
    }
    const CT t3 = (P[0] + P[1] + P[2]) * (CT)(1.0 / 3.0);
    const CT P2xy = (CT)2 * P[3], P2xz = (CT)2 * P[4], P2yz = (CT)2 * P[5];
    const CT keep = (CT)1 - omg;
    n[0] = w0 * a + keep * ne0 - (CT)1.5 * w0 * 3 * (g1 + g2) * t3;
#pragma unroll
    for (int pi = 0; pi < 9; ++pi) {
      const int q = 2 * pi + 1, b = q + 1;
      const CT cu = cdot<CT>(q, ux, uy, uz);
      const CT sym = fmaT(q <= 6 ? b1 : b2, cu * cu, q <= 6 ? a1 : a2);
      const CT anti = (q <= 6 ? c1 : c2) * cu;
      CT pcc = (cx(q) != 0 ? P[0] : (CT)0) + (cy(q) != 0 ? P[1] : (CT)0) + (cz(q) != 0 ? P[2] : (CT)0);
      addc(pcc, cx(q) * cy(q), P2xy);  // Pi : c c = sum_a Pi_aa c_a^2 + 2 sum_a<b Pi_ab c_a c_b
      addc(pcc, cx(q) * cz(q), P2xz);
      addc(pcc, cy(q) * cz(q), P2yz);
      const int c2q = cx(q) * cx(q) + cy(q) * cy(q) + cz(q) * cz(q);
      const CT Q = (CT)4.5 * (q <= 6 ? w1 : w2) * (g1 * (pcc - t3) + g2 * t3 * (CT)(c2q - 1));
      n[q] = (sym + anti) + fmaT(keep, n[q], Q);
      n[b] = (sym - anti) + fmaT(keep, n[b], Q);
    }
  }
  // non-equilibrium momentum flux Pi^neq = sum_q (n_q - feq_q) c_q c_q (pairs add), the
  // node's mass deviation and the fluid node count
#pragma unroll
  for (int pi = 0; pi < 9; ++pi) {
    const int q = 2 * pi + 1;
    if (cx(q) != 0) pacc[0] += ps[pi];
    if (cy(q) != 0) pacc[1] += ps[pi];
    if (cz(q) != 0) pacc[2] += ps[pi];
    addc(pacc[3], cx(q) * cy(q), ps[pi]);
    addc(pacc[4], cx(q) * cz(q), ps[pi]);
    addc(pacc[5], cy(q) * cz(q), ps[pi]);
  }
  pacc[6] += rd;
  pacc[7] += (CT)1;
  }
  if (xin) {
    uint32_t sb = rowc + (uint32_t)x * es;
    asm volatile("" : "+v"(sb));
#pragma unroll
    for (int q = 0; q < NQ; ++q) RowIO<ST>::st_stream(rout, q * pb + sb, n[q], q, A.h16);
  }
}

template <class ST, int COLL>
__global__ __launch_bounds__(256, (sizeof(ST) <= 4 && COLL == 0) ? 8 : 1) void k_stream(StreamArgs A) {
  using CT = typename Store<ST>::CT;
  __shared__ CT spn[NPIN][256];  // per-thread partials of the fluid stress and mass
  const int brick = (blockIdx.x & 7) * A.per_xcd + (blockIdx.x >> 3);
  if (brick >= A.nbricks) return;  // the whole work-group
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int lx = A.lx, ly = A.ly, lz = A.lz;
  const int bxi = brick % A.bxn, byi = (brick / A.bxn) % A.byn, bzi = brick / (A.bxn * A.byn);
  const int x0 = bxi * TX + lane;
  const bool xin = x0 < lx;
  const int y_lo = byi * A.BY, y_hi = min(ly, y_lo + A.BY);
  const int z_lo = bzi * A.BZ, z_hi = min(lz, z_lo + A.BZ);
  constexpr uint32_t es = sizeof(ST);
  const uint32_t pb0 = (uint32_t)(A.plane * es);  // plane stride in bytes
  const __amdgpu_buffer_rsrc_t rin = buf_rsrc(A.fin, A.pop_bytes), rout = buf_rsrc(A.fout, A.pop_bytes);
  const __amdgpu_buffer_rsrc_t rgh = buf_rsrc(A.gval, A.gval_bytes), rrec = buf_rsrc(A.lrec, A.rec_bytes);
  CT pacc[NPIN];
#pragma unroll
  for (int c = 0; c < NPIN; ++c) pacc[c] = 0;
  uint32_t bad = 0;  // flags raised by this lane
  uint32_t nfast = 0;  // fluid nodes of this lane above 0.3 c_s
  CT umax = 0;         // their largest u^2
  // link record of (x0, y, z) and the first link value of its row; a lane past the box end
  // reads as solid
  auto record = [&](int y, int z) -> uint32_t {
    return xin ? __builtin_amdgcn_raw_buffer_load_b32(rrec, (uint32_t)(x0 + lx * (y + ly * z)) * 4u, 0, 0)
               : REC_SOLID;
  };
  auto rowv = [&](int y, int z) -> uint32_t { return A.vbase + (uint32_t)A.lrow[(z * ly + y) * A.bxn + bxi]; };
#pragma unroll 1
  for (int yb = y_lo + wv; yb < y_hi; yb += 4) {
    uint32_t rnext = record(yb, z_lo), vnext = rowv(yb, z_lo);
#pragma unroll 1
    for (int zb = z_lo; zb < z_hi; ++zb) {
      const int y = opaque_uniform(yb), z = opaque_uniform(zb);
      const uint32_t pb = (uint32_t)opaque_uniform((int)pb0);
      // the lane's column, made opaque here so that what derives from it is formed in the
      // loop instead of being kept across it
      int x = x0;
      asm volatile("" : "+v"(x));
      const uint32_t rec = rnext, vrow = vnext;
      if (zb + 1 < z_hi) {  // the next node's record, a step ahead
        rnext = record(y, z + 1);
        vnext = rowv(y, z + 1);
      }
      stream_node<ST, COLL, 0>(A, rin, rout, rgh, pb, x, y, z, xin, rec, vrow, pacc, bad, nfast, umax,
                               LinkSlots<CT>{});
    }
  }
  stream_tail<CT>(A, brick, spn, pacc, bad, nfast, umax);
}

// ---- k_lattice: the links and the stream of one 64 x 4 x 4 brick in one work-group: list and
// table, pre (link corrections into the slots), stream (wave w streams row y0 + w through the
// brick's z-slices), sums.  The slots past VLDS and the records of the list stay within the
// work-group (a barrier apart; the slots' global overflow block is the brick's own). ----
struct LatticeArgs {
  LinksArgs L;
  StreamArgs S;
};

// pre, stream, sums of a brick (OVF: the brick has more links than the LDS slots)
template <class ST, int COLL, bool OVF>
__device__ __forceinline__ void lattice_rest(const LatticeArgs &P, int brick, LinksLDS &sh,
                                             const LinkSlots<typename Store<ST>::CT> &S, int cnt, uint32_t bad) {
  using CT = typename Store<ST>::CT;
  lattice_pre<ST, OVF>(P.L, brick, sh, S, cnt);
  __syncthreads();  // the corrections in their slots
  const StreamArgs &A = P.S;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int lx = A.lx, ly = A.ly, lz = A.lz;
  const int x0 = (brick % A.bxn) * LBX, y0 = ((brick / A.bxn) % A.byn) * LBY, z0 = (brick / (A.bxn * A.byn)) * LBZ;
  const int nsl = min(LBZ, lz - z0);
  constexpr uint32_t es = sizeof(ST);
  const uint32_t pb = (uint32_t)opaque_uniform((int)(A.plane * es));
  const __amdgpu_buffer_rsrc_t rin = buf_rsrc(A.fin, A.pop_bytes), rout = buf_rsrc(A.fout, A.pop_bytes);
  const __amdgpu_buffer_rsrc_t rgh = buf_rsrc(A.gval, A.gval_bytes);
  CT pacc[NPIN];
#pragma unroll
  for (int c = 0; c < NPIN; ++c) pacc[c] = 0;
  uint32_t nfast = 0;
  CT umax = 0;
  const int x = x0 + lane;
  const bool xin = x < lx;
  if (y0 + wv < ly) {
#pragma unroll 1
    for (int sl = 0; sl < nsl; ++sl) {
      const int loc = lane | (wv << 6) | (sl << 8);
      stream_node<ST, COLL, OVF ? 2 : 1>(A, rin, rout, rgh, pb, x, opaque_uniform(y0 + wv), opaque_uniform(z0 + sl),
                                         xin, sh.srec[loc], sh.srow[wv + LBY * sl], pacc, bad, nfast, umax, S);
    }
  }
  if (nfast) {  // rare: the health counters (count of fast node-steps, largest u^2 as bits)
    atomicAdd((unsigned long long *)(A.flags + FL_HEALTH), (unsigned long long)nfast);
    atomicMax(A.flags + FL_HEALTH + 2, __float_as_int((float)umax));
  }
  // the brick's partials of the fluid stress and mass: each wave's lanes by a fixed butterfly,
  // then the four waves in order
#pragma unroll
  for (int c = 0; c < NPIN; ++c) {
    const double v = wave_sum((double)pacc[c]);
    if (lane == 0) sh.spw[wv][c] = v;
  }
  __syncthreads();  // the slots hold n*_qbar(X); the partials are in
  if (threadIdx.x < NPIN) {
    const int c = threadIdx.x;
    A.pin[(size_t)brick * NPIN + c] = (sh.spw[0][c] + sh.spw[1][c]) + (sh.spw[2][c] + sh.spw[3][c]);
  }
  lattice_sums<ST, OVF>(P.L, brick, sh, S, cnt, bad);
}

// bid: the work-group's index among its simulation's (a multiple of 8 apart from blockIdx.x
// in multi-job launches, so the XCD of a brick is the same as in a launch of its own)
template <class ST, int COLL>
__device__ __forceinline__ void lattice_wg(const LatticeArgs &P, const int bid) {
  using CT = typename Store<ST>::CT;
  __shared__ LinksLDS sh;
  __shared__ CT sval[VLDS + 64];  // the slots and the lanes' spare slots
  const int brick = (bid & 7) * P.L.per_xcd + (bid >> 3);
  if (brick >= P.L.nbricks) return;  // the whole work-group
  if (threadIdx.x < 64) sval[VLDS + threadIdx.x] = (CT)0;
  uint32_t bad = 0;
  const int cnt = links_list<ST, true>(P.L, brick, sh, bad);  // (its barriers order the spares' zeros)
  constexpr uint32_t es = sizeof(ST);
  LinkSlots<CT> S;
  S.lds = sval;
  S.r = buf_rsrc(P.L.f, P.L.pop_bytes);
  S.block = (P.L.vbase + (uint32_t)brick * BRICK_VALUES) * es;
  S.ovf = __builtin_amdgcn_readfirstlane(sh.vcount) > VLDS;
  if (S.ovf) lattice_rest<ST, COLL, true>(P, brick, sh, S, cnt, bad);
  else lattice_rest<ST, COLL, false>(P, brick, sh, S, cnt, bad);
}

template <class ST, int COLL>
__global__ __launch_bounds__(256, sizeof(ST) <= 4 ? 4 : 1) void k_lattice(LatticeArgs P) {
  lattice_wg<ST, COLL>(P, (int)blockIdx.x);
}
template <class ST, int COLL>
__global__ __launch_bounds__(256, sizeof(ST) <= 4 ? 4 : 1) void k_lattice_m(const LatticeArgs *__restrict__ tab,
                                                                        const int32_t *__restrict__ pre, int nj) {
  SUSP_MULTI_BODY(LatticeArgs, (lattice_wg<ST, COLL>));
}

static uint32_t pop_bytes(const Sim *s) {  // the populations and the link values after them
  const size_t es = s->precision == 0 ? 8 : s->precision == 1 ? 4 : 2;
  return (uint32_t)((NQ * s->plane + link_values(s->lx, s->ly, s->lz)) * es);  // < 2^32, checked at creation
}
static uint32_t gval_bytes(const Sim *s) {
  const size_t ges = s->precision == 0 ? 8 : 4;
  return (uint32_t)(10 * (size_t)s->lx * s->lz * ges);
}

static LinksArgs links_args(const Sim *s, const Box &b) {
  LinksArgs A;
  A.f = s->f[s->cur];
  A.plane = s->plane;
  A.pop_bytes = pop_bytes(s);
  A.goff = (int)(s->gown - s->own);
  A.ow_bytes = (uint32_t)(((size_t)A.goff + 2 * (size_t)s->lx * s->lz) * 4);
  A.own = s->own;
  A.lrec = s->lrec;
  A.lrow = s->lrow;
  A.vbase = (uint32_t)(NQ * s->plane);
  A.vcap = (uint32_t)link_values(s->lx, s->ly, s->lz);
  A.R = s->R[s->pcur]; A.U = s->U[s->pcur]; A.W = s->W[s->pcur];
  A.hacc = s->hacc;
  A.flags = s->flags;
  A.lx = s->lx; A.ly = s->ly; A.lz = s->lz;
  A.bxn = (s->lx + LBX - 1) / LBX;
  A.byn = (s->ly + LBY - 1) / LBY;
  A.nbricks = A.bxn * A.byn * ((s->lz + LBZ - 1) / LBZ);
  A.per_xcd = (A.nbricks + 7) / 8;
  A.b = b;
  A.clk = s->clk;
  A.kax = -6.0 * wq(1) * s->rho0;
  A.kdg = -6.0 * wq(7) * s->rho0;
  A.h16 = s->h16;
  return A;
}

static StreamArgs stream_args(const Sim *s) {
  StreamArgs A;
  A.fin = s->f[s->cur];
  A.fout = s->f[1 - s->cur];
  A.plane = s->plane;
  A.pop_bytes = pop_bytes(s);
  A.gval_bytes = gval_bytes(s);
  A.rec_bytes = (uint32_t)(s->nodes * 4);
  A.lrec = s->lrec;
  A.lrow = s->lrow;
  A.vbase = (uint32_t)(NQ * s->plane);
  A.gval = s->gval;
  A.pin = s->pin;
  A.flags = s->flags;
  A.lx = s->lx; A.ly = s->ly; A.lz = s->lz;
  A.bxn = s->bxn; A.byn = s->byn; A.BY = s->BY; A.BZ = s->BZ;
  A.nbricks = s->nbricks;
  A.per_xcd = (s->nbricks + 7) / 8;
  A.rho0 = s->rho0;
  A.omega = 1.0 / s->tau;
  A.om_ghost = 1.0 / s->tau_ghost;
  A.om_bulk = 1.0 / s->tau_bulk;
  A.h16 = s->h16;
  return A;
}

// Whether the step runs k_lattice (links and stream of a brick in one work-group): the stream
// bricks are the link bricks (64 x 4 x 4) and there are spheres.
static bool fused(const Sim *s) { return s->n > 0 && s->BY == LBY && s->BZ == LBZ; }

// The links (k_links, or k_lattice): after the ghost planes, before k_stream.
hipError_t launch_links(Sim *s, const Box &b) {
  if (s->n == 0) return hipSuccess;
  if (fused(s)) {
    LatticeArgs P;
    P.L = links_args(s, b);
    P.L.lrec = nullptr;  // the stream phase takes the records from LDS
    P.L.lrow = nullptr;
    P.S = stream_args(s);
    const unsigned grid = P.L.per_xcd * 8;
    if (s->collision == 0) {
      if (s->precision == 0) return dispatch(s, k_lattice<double, 0>, k_lattice_m<double, 0>, grid, 256, P);
      if (s->precision == 1) return dispatch(s, k_lattice<float, 0>, k_lattice_m<float, 0>, grid, 256, P);
      return dispatch(s, k_lattice<__half, 0>, k_lattice_m<__half, 0>, grid, 256, P);
    }
    if (s->precision == 0) return dispatch(s, k_lattice<double, 1>, k_lattice_m<double, 1>, grid, 256, P);
    if (s->precision == 1) return dispatch(s, k_lattice<float, 1>, k_lattice_m<float, 1>, grid, 256, P);
    return dispatch(s, k_lattice<__half, 1>, k_lattice_m<__half, 1>, grid, 256, P);
  }
  SUSP_NO_COLLECT(s);
  const LinksArgs A = links_args(s, b);
  const dim3 grid(A.per_xcd * 8), blk(256);
  if (s->precision == 0) hipLaunchKernelGGL(k_links<double>, grid, blk, 0, s->stream, A);
  else if (s->precision == 1) hipLaunchKernelGGL(k_links<float>, grid, blk, 0, s->stream, A);
  else hipLaunchKernelGGL(k_links<__half>, grid, blk, 0, s->stream, A);
  return hipGetLastError();
}

// The streaming kernel (k_stream): pull, collision, partials (nothing when k_lattice ran).
hipError_t launch_lbm(Sim *s, const Box &b) {
  (void)b;
  if (fused(s)) return hipSuccess;
  SUSP_NO_COLLECT(s);
  const StreamArgs A = stream_args(s);
  dim3 grid(A.per_xcd * 8), blk(256);
  if (s->collision == 0) {
    if (s->precision == 0) hipLaunchKernelGGL((k_stream<double, 0>), grid, blk, 0, s->stream, A);
    else if (s->precision == 1) hipLaunchKernelGGL((k_stream<float, 0>), grid, blk, 0, s->stream, A);
    else hipLaunchKernelGGL((k_stream<__half, 0>), grid, blk, 0, s->stream, A);
  } else {
    if (s->precision == 0) hipLaunchKernelGGL((k_stream<double, 1>), grid, blk, 0, s->stream, A);
    else if (s->precision == 1) hipLaunchKernelGGL((k_stream<float, 1>), grid, blk, 0, s->stream, A);
    else hipLaunchKernelGGL((k_stream<__half, 1>), grid, blk, 0, s->stream, A);
  }
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
  Box b;             // with clk set, offset and velocity come from the clock
  const Clock *clk;
  int lx, ly, lz, n;
  double rho0;
  int values;
  int32_t *gown;
  int32_t *gcnt;  // spheres covering each ghost point
  void *gval;
  int32_t *flags;
  H16 h16;
};

// Galilean-corrected post-collision deviations of the five directions of ghost plane G at
// node (x,yrow,z) seen from the neighbouring image box: sgn = +1 box below (u - ule), -1 box
// above (u + ule).  The node's moments are formed once for the five.
template <int G, class ST, class CT>
__device__ inline void nhat5(const ST *fin, size_t plane, const int32_t *own, const double *R,
                             const double *U, const double *W, Box b, double rho0, H16 h16, int x,
                             int yrow, int z, int sgn, CT out[5]) {
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
    const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      const int q = gdir(G, m);
      const double cu = cx(q) * ux + cy(q) * uy + cz(q) * uz;
      out[m] = (CT)(wq(q) * rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
    }
    return;
  }
  CT rd = 0, jx = 0, jy = 0, jz = 0, fq[5];
#pragma unroll
  for (int r = 0; r < NQ; ++r) {
    const CT v = Store<ST>::ld(fin, (size_t)r * plane + node, r, h16);
    rd += v; jx += v * (CT)cx(r); jy += v * (CT)cy(r); jz += v * (CT)cz(r);
#pragma unroll
    for (int m = 0; m < 5; ++m)
      if (r == gdir(G, m)) fq[m] = v;
  }
  const CT rho = (CT)rho0 + rd;
  const CT ux = jx / rho, uy = jy / rho, uz = jz / rho;
  // feq(rho, u + du) - feq(rho, u) with du = -sgn ule x, written out to avoid cancellation
  const CT du = (CT)(-sgn * b.ule);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    const int q = gdir(G, m);
    const CT cu = (CT)cx(q) * ux + (CT)cy(q) * uy + (CT)cz(q) * uz;
    const CT cd = (CT)cx(q) * du;
    const CT dfe = (CT)wq(q) * rho * ((CT)3 * cd + (CT)4.5 * cd * ((CT)2 * cu + cd) -
                                      (CT)1.5 * du * ((CT)2 * ux + du));
    out[m] = fq[m] + dfe;
  }
}

// Values of ghost plane G at (x, z): the row of the neighbouring image interpolated linearly
// at the sheared position.
template <int G, class ST, class CT>
__device__ inline void ghost_values(const GhostArgs &A, const Box &bx, int x, int z) {
  const ST *fin = (const ST *)A.fin;
  CT *gval = (CT *)A.gval;
  const int sgn = G == 0 ? 1 : -1;
  const int yrow = G == 0 ? A.ly - 1 : 0;
  const double xs = (double)x + sgn * bx.s;
  const double x0f = floor(xs);
  const double fr = xs - x0f;
  int i0 = (int)x0f % A.lx;
  i0 = i0 < 0 ? i0 + A.lx : i0;
  const int i1 = i0 + 1 == A.lx ? 0 : i0 + 1;
  CT v0[5], v1[5];
  nhat5<G, ST, CT>(fin, A.plane, A.own, A.R, A.U, A.W, bx, A.rho0, A.h16, i0, yrow, z, sgn, v0);
  nhat5<G, ST, CT>(fin, A.plane, A.own, A.R, A.U, A.W, bx, A.rho0, A.h16, i1, yrow, z, sgn, v1);
#pragma unroll
  for (int m = 0; m < 5; ++m)
    gval[(size_t)((G * 5 + m) * A.lz + z) * A.lx + x] = ((CT)1 - (CT)fr) * v0[m] + (CT)fr * v1[m];
}

// Ghost owners by footprint: a wave per sphere; each image of the sphere within reach of a
// ghost plane visits the ghost points of its footprint there and applies the geometric test
// (minimum image, squared distance below the mapped radius squared).  A covered point takes
// the smallest id (the owners start at INT32_MAX; k_ghost_values marks uncovered points -1);
// the count of spheres covering it finds overlaps.  Each point is visited at
// most once per sphere: only through the image the minimum image picks, and the footprint
// ranges are taken modulo the box without repeats.
__device__ inline void ghost_range(double c, double r, int L, int &lo, int &cnt) {
  int a = (int)ceil(c - r - 1e-6), b = (int)floor(c + r + 1e-6);
  if (b - a + 1 >= L) { a = 0; b = L - 1; }
  lo = a;
  cnt = b - a + 1;
}
__device__ __forceinline__ void ghost_raster_wg(const GhostArgs &A, const int bid) {
  const Box bx = clock_box(A.b, A.clk, 0);
  const int p = bid * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (p >= A.n) return;  // the whole wave
  const double Rx = A.R[3 * p], Ry = A.R[3 * p + 1], Rz = A.R[3 * p + 2], am = A.amap[p];
  if (!(isfinite(Rx) && isfinite(Ry) && isfinite(Rz))) return;  // covers nothing (the step reports it)
  const double am2 = am * am;
#pragma unroll 1
  for (int g = 0; g < 2; ++g) {
    const double gy = g == 0 ? -1.0 : (double)A.ly;
#pragma unroll 1
    for (int k = -1; k <= 1; ++k) {
      // the image at (Rx + k s, Ry + k Ly); a margin of one node keeps the rounding of the
      // minimum image inside the footprint
      if (!(fabs(gy - (Ry + k * bx.Ly)) < am + 1.0)) continue;
      int xa, nx, za, nz;
      ghost_range(Rx + k * bx.s, am + 1.0, A.lx, xa, nx);
      ghost_range(Rz, am + 1.0, A.lz, za, nz);
      const int tot = nx * nz;
      for (int t = lane; t < tot; t += 64) {
        const int iz = t / nx, ix = t - iz * nx;
        int x = (xa + ix) % A.lx;
        x = x < 0 ? x + A.lx : x;
        int z = (za + iz) % A.lz;
        z = z < 0 ? z + A.lz : z;
        double dx, dy, dz;
        int kk;
        minimage(bx, (double)x - Rx, gy - Ry, (double)z - Rz, dx, dy, dz, kk);
        if (kk != k) continue;
        if (dx * dx + dy * dy + dz * dz < am2) {
          const int pt = (g * A.lz + z) * A.lx + x;
          atomicMin(&A.gown[pt], p);
          atomicAdd(&A.gcnt[pt], 1);
        }
      }
    }
  }
}
__global__ __launch_bounds__(256) void k_ghost_raster(GhostArgs A) { ghost_raster_wg(A, (int)blockIdx.x); }
__global__ __launch_bounds__(256) void k_ghost_raster_m(const GhostArgs *__restrict__ tab,
                                                        const int32_t *__restrict__ pre, int nj) {
  SUSP_MULTI_BODY(GhostArgs, ghost_raster_wg);
}

// One thread per ghost point: -1 where no sphere covers it, an overlap where two do, and
// (fluid points) the values.
template <class ST>
__device__ __forceinline__ void ghost_values_wg(const GhostArgs &A, const int bid) {
  using CT = typename Store<ST>::CT;
  const Box bx = clock_box(A.b, A.clk, 0);
  const int idx = bid * 256 + threadIdx.x;
  const int npl = A.lx * A.lz;
  if (idx >= 2 * npl) return;
  const int cover = A.gcnt[idx];
  if (cover == 0) A.gown[idx] = -1;
  if (cover > 1) atomicOr(A.flags, 1);
  if (!A.values || cover > 0) return;
  const int g = idx / npl;
  const int rem = idx - g * npl;
  const int z = rem / A.lx, x = rem - z * A.lx;
  if (g == 0) ghost_values<0, ST, CT>(A, bx, x, z);
  else ghost_values<1, ST, CT>(A, bx, x, z);
}
template <class ST>
__global__ __launch_bounds__(256) void k_ghost_values(GhostArgs A) { ghost_values_wg<ST>(A, (int)blockIdx.x); }
template <class ST>
__global__ __launch_bounds__(256) void k_ghost_values_m(const GhostArgs *__restrict__ tab,
                                                        const int32_t *__restrict__ pre, int nj) {
  SUSP_MULTI_BODY(GhostArgs, ghost_values_wg<ST>);
}

__global__ __launch_bounds__(256) void k_ghost_clear(int32_t *gown, int32_t *gcnt, int npts) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < npts) { gown[i] = 0x7fffffff; gcnt[i] = 0; }
}

hipError_t launch_ghosts(Sim *s, const Box &b, int32_t *gown_out, int32_t *gcnt, void *gval_out, int values,
                         const Clock *clk, int cleared) {
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
  A.clk = clk;
  A.lx = s->lx; A.ly = s->ly; A.lz = s->lz; A.n = s->n;
  A.rho0 = s->rho0;
  A.values = values;
  A.gown = gown_out;
  A.gcnt = gcnt;
  A.gval = gval_out;
  A.flags = s->flags;
  A.h16 = s->h16;
  const int tot = 2 * s->lx * s->lz;
  const unsigned grid = (tot + 255) / 256;
  if (!cleared) {
    SUSP_NO_COLLECT(s);
    hipLaunchKernelGGL(k_ghost_clear, dim3(grid), dim3(256), 0, s->stream, gown_out, gcnt, tot);
  }
  hipError_t e = hipSuccess;
  if (s->n > 0) e = dispatch(s, k_ghost_raster, k_ghost_raster_m, (s->n + 3) / 4, 256, A);
  if (e != hipSuccess) return e;
  if (s->precision == 0) return dispatch(s, k_ghost_values<double>, k_ghost_values_m<double>, grid, 256, A);
  if (s->precision == 1) return dispatch(s, k_ghost_values<float>, k_ghost_values_m<float>, grid, 256, A);
  return dispatch(s, k_ghost_values<__half>, k_ghost_values_m<__half>, grid, 256, A);
}

// ---------------------------------------------------------------------------------------
// Moving walls (boundary 1, Sec. 3): flat walls halfway between the edge rows and their
// ghost planes, moving at -uw (bottom) and +uw (top) in x.  The ghost value pulled along q
// by the edge node X = (x + c_qx, edge row, z + c_qz) is that node's own opposite
// population plus the wall's momentum (eq. 7): d_q = d_qbar(X) + 6 w_q rho0 u_w c_qx, so the
// lattice kernel needs no change.  Each block also sums the momentum the walls receive from
// fluid edge nodes, -(2 d_qbar + 6 w_q rho0 u_w c_qx) c_q (measured from the rest state).
template <class ST>
__global__ __launch_bounds__(256) void k_walls(const void *fin, size_t plane, const int32_t *own, int lx,
                                               int ly, int lz, double rho0, H16 h16, const Clock *clk,
                                               int32_t *gown, void *gval, double *wpart) {
  using CT = typename Store<ST>::CT;
  __shared__ double red[6][256];
  const int t = threadIdx.x;
  const int idx = blockIdx.x * blockDim.x + t;
  const int npl = lx * lz;
  double mom[6] = {0, 0, 0, 0, 0, 0};
  if (idx < 2 * npl) {
    const int g = idx / npl;
    const int rem = idx - g * npl;
    const int z = rem / lx, x = rem - (rem / lx) * lx;
    const double uw = g == 0 ? -clk->cur.uw : clk->cur.uw;
    const int yrow = g == 0 ? 0 : ly - 1;
    gown[idx] = -1;
    CT *gv = (CT *)gval;
    for (int m = 0; m < 5; ++m) {
      const int q = gdir(g, m), qb = opp(q);
      int xs = x + cx(q), zs = z + cz(q);
      xs = xs < 0 ? xs + lx : (xs >= lx ? xs - lx : xs);
      zs = zs < 0 ? zs + lz : (zs >= lz ? zs - lz : zs);
      const int64_t node = xs + (int64_t)lx * (yrow + (int64_t)ly * zs);
      const CT d = Store<ST>::ld((const ST *)fin + (size_t)qb * plane, node, qb, h16);
      const double mw = 6.0 * wq(q) * rho0 * uw * cx(q);
      gv[(size_t)((g * 5 + m) * lz + z) * lx + x] = d + (CT)mw;
      if (own[node] == -1) {
        const double mm = 2.0 * (double)d + mw;
        mom[3 * g] -= mm * cx(q);
        mom[3 * g + 1] -= mm * cy(q);
        mom[3 * g + 2] -= mm * cz(q);
      }
    }
  }
  for (int c = 0; c < 6; ++c) red[c][t] = mom[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
      for (int c = 0; c < 6; ++c) red[c][t] += red[c][t + w];
    __syncthreads();
  }
  if (t < 6) wpart[(size_t)blockIdx.x * 6 + t] = red[t][0];
}

hipError_t launch_walls(Sim *s) {
  SUSP_NO_COLLECT(s);
  const int tot = 2 * s->lx * s->lz;
  dim3 grid((tot + 255) / 256), blk(256);
  if (s->precision == 0)
    hipLaunchKernelGGL(k_walls<double>, grid, blk, 0, s->stream, s->f[s->cur], s->plane, s->own, s->lx, s->ly,
                       s->lz, s->rho0, s->h16, s->clk, s->gown, s->gval, s->wpart);
  else if (s->precision == 1)
    hipLaunchKernelGGL(k_walls<float>, grid, blk, 0, s->stream, s->f[s->cur], s->plane, s->own, s->lx, s->ly,
                       s->lz, s->rho0, s->h16, s->clk, s->gown, s->gval, s->wpart);
  else
    hipLaunchKernelGGL(k_walls<__half>, grid, blk, 0, s->stream, s->f[s->cur], s->plane, s->own, s->lx, s->ly,
                       s->lz, s->rho0, s->h16, s->clk, s->gown, s->gval, s->wpart);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Start of a step: the table entry of the step becomes the current clock (reset: rewind the
// cursor after a new table upload).
// The clock of the step (thread 0), and the cleared ghost owner planes for k_ghost_raster
// (gown: no owner yet, INT32_MAX; gcnt: no cover), so that the step needs no launch for them.
struct ClockArgs {
  const ClockEntry *tab;
  Clock *clk;
  int reset;
  int32_t *gown, *gcnt;
  int npts;
};
__device__ __forceinline__ void clock_wg(const ClockArgs &A, const int bid) {
  const int g = bid * 256 + threadIdx.x;
  if (g < A.npts) { A.gown[g] = 0x7fffffff; A.gcnt[g] = 0; }
  if (g != 0) return;
  if (A.reset) {
    A.clk->idx = 0;
    return;
  }
  const int i = A.clk->idx;
  A.clk->cur = A.tab[i < CLK_CAP ? i : CLK_CAP - 1];
  A.clk->idx = i + 1;
}
__global__ __launch_bounds__(256) void k_clock(ClockArgs A) { clock_wg(A, (int)blockIdx.x); }
__global__ __launch_bounds__(256) void k_clock_m(const ClockArgs *__restrict__ tab, const int32_t *__restrict__ pre,
                                                 int nj) {
  SUSP_MULTI_BODY(ClockArgs, clock_wg);
}

hipError_t launch_clock(Sim *s, int reset) {
  // the step's ghost planes are cleared here (Lees-Edwards steps)
  ClockArgs A;
  A.tab = s->clk_tab;
  A.clk = s->clk;
  A.reset = reset;
  A.gown = s->gown;
  A.gcnt = s->gcnt;
  A.npts = !reset && s->boundary == 0 ? 2 * s->lx * s->lz : 0;
  return dispatch(s, k_clock, k_clock_m, A.npts > 0 ? (A.npts + 255) / 256 : 1, 256, A);
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

// One plane q: FP64 full values <-> storage deviations of the current state.
// (Solid nodes read as the rest state: the lattice kernel keeps no populations there.)
template <class ST>
__global__ void k_pop_plane(void *fv, double *d64, const int32_t *own, size_t plane, int64_t nodes, int q,
                            double rho0, int to_storage, H16 h16) {
  using CT = typename Store<ST>::CT;
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= nodes) return;
  ST *f = (ST *)fv + (size_t)q * plane;
  const double w = wq(q) * rho0;
  if (to_storage) Store<ST>::st(f, node, (CT)(d64[node] - w), q, h16);
  else d64[node] = own[node] >= 0 ? w : w + (double)Store<ST>::ld(f, node, q, h16);
}

hipError_t launch_pop_plane(Sim *s, double *dev64, int q, int to_storage) {
  dim3 grid((unsigned)((s->nodes + 255) / 256)), blk(256);
  void *f = s->f[s->cur];
  if (s->precision == 0)
    hipLaunchKernelGGL(k_pop_plane<double>, grid, blk, 0, s->stream, f, dev64, s->own, s->plane, s->nodes, q, s->rho0, to_storage, s->h16);
  else if (s->precision == 1)
    hipLaunchKernelGGL(k_pop_plane<float>, grid, blk, 0, s->stream, f, dev64, s->own, s->plane, s->nodes, q, s->rho0, to_storage, s->h16);
  else
    hipLaunchKernelGGL(k_pop_plane<__half>, grid, blk, 0, s->stream, f, dev64, s->own, s->plane, s->nodes, q, s->rho0, to_storage, s->h16);
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

// Link owners of direction q: for every node, the owner of its pull source x - c_q (map or
// ghost plane) if the node is fluid and the source solid, else -1.
__global__ void k_link_enum(const int32_t *own, const int32_t *gown, int64_t nodes, int lx,
                            int ly, int lz, int q, int32_t *out) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= nodes) return;
  const int x = (int)(node % lx);
  const int64_t yz = node / lx;
  const int y = (int)(yz % ly), z = (int)(yz / ly);
  int so = -1;
  if (own[node] < 0) {
    int px = x - cx(q), py = y - cy(q), pz = z - cz(q);
    px = px < 0 ? px + lx : (px >= lx ? px - lx : px);
    pz = pz < 0 ? pz + lz : (pz >= lz ? pz - lz : pz);
    if (py < 0 || py >= ly) so = gown[((py < 0 ? 0 : 1) * lz + pz) * lx + px];
    else so = own[px + (int64_t)lx * (py + (int64_t)ly * pz)];
    if (so < 0) so = -1;
  }
  out[node] = so;
}

hipError_t launch_link_enum(Sim *s, const int32_t *gown, int32_t *out, int q) {
  dim3 grid((unsigned)((s->nodes + 255) / 256)), blk(256);
  hipLaunchKernelGGL(k_link_enum, grid, blk, 0, s->stream, s->own, gown, s->nodes,
                     s->lx, s->ly, s->lz, q, out);
  return hipGetLastError();
}

}  // namespace susp
