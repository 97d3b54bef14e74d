// fluid.hip -- lattice-Boltzmann kernels for gfx950.
//
//  k_lbm      fused pull-stream + moving bounce-back + BGK collision + link forces + fluid
//             stress partials (App. A eqs. 3-10), one thread per node, x fastest.
//  k_ghosts   Lees-Edwards ghost planes y=-1 and y=ly: geometric owner test of each ghost
//             point, else linear interpolation of the Galilean-corrected post-collision
//             row shifted by the offset (Wagner & Pagonabarraga).
//  helpers    equilibrium fill, FP64 <-> storage conversion, link enumeration.
#include "susp_impl.h"

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
// Lattice kernel k_lbm: pull-stream, moving bounce-back, link sums, BGK collision and the
// fluid stress partials in one pass.  The lattice is walked in bricks of TX x BY x BZ
// nodes, one work-group per brick: its four waves take four consecutive rows (one 64-node
// x segment each) and walk the brick's z range together.  The owner map of planes z-1 ..
// z+2 (rows y-1 .. y+4 with a one-node x halo; rows beyond the box edges come from the
// Lees-Edwards ghost owner planes) sits in a ring of five LDS planes; each z step fetches
// plane z+3.  Row and plane of every pull source are uniform over a wave, so a population
// load is a uniform row offset plus the lane's (periodically wrapped) x.  The spheres that
// can own a node of the brick's staged region are listed per brick beforehand
// (k_brick_lists); their states sit in LDS beside the brick's link table.
//
// Links: with lever r_b - R = D - c_q/2 (D = node minus sphere centre, minimum image) the
// surface velocity along the link is u_b.c_q = u(X).c_q, because (W x c).c = 0; hence one
// FP64 minimum image and one rigid-body velocity per node and sphere, and per link only
//   corr = -6 w_q rho0 u(X).c_q,  n_q = n*_qbar - corr,  m = 2 n*_qbar - corr.
// The node's sums are F = -sum m c_q, T = D x F, S = sym(D (x) F) + 1/2 sum m c_q c_q
// (exactly the link sums of eqs. 6, 9, 10 regrouped).  A sphere is convex, so of two
// opposite directions at most one links the node to the same sphere; the sums are formed
// per opposite pair, in FP64 (torque and stresslet cancel strongly over a surface).
// Per-sphere sums of the brick are accumulated in an LDS hash table with one copy per wave
// (a wave adds its lanes in a fixed order; the copies are summed in wave order) and written
// once per brick; k_hydro_gather adds a sphere's brick entries in a fixed order.  The sums
// are therefore bitwise reproducible (unless more than TSLOT spheres are listed for a
// brick: the rest go through global atomics).
constexpr int TX = 64, TY = 4;
constexpr int TSLOT = 128;
constexpr int SDAT = 10;  // doubles per LDS sphere state (R, U, W; padded to 16 bytes)
constexpr int SPCAP = 64;  // table entries with links kept per sphere (past it: enumeration)
static_assert(SPCAP == 64, "k_hydro_gather reads a sphere's entry slots with one wave");
constexpr int SROW = TX + 2, SPLANE = (TY + 2) * SROW;  // staged owner plane: 6 rows of 66

struct LbmArgs {
  const void *fin;
  void *fout;
  size_t plane;
  uint32_t pop_bytes, gval_bytes;  // bytes of one population array (< 4 GiB), of gval
  const int32_t *own;
  const int32_t *gown;
  const void *gval;
  const double *R, *U, *W;
  int32_t *bt_key;        // in: the spheres listed for each brick; out: its table's keys
  const int32_t *bt_cnt;  // number of spheres listed for each brick
  double *bt_val;
  int32_t *sp_cnt, *sp_ent;  // per sphere: its table entries with links (brick*TSLOT+slot)
  double *hyd_fb;
  double *pineq;
  int32_t *flags;
  int lx, ly, lz;
  int bxn, byn, bzn, BY, BZ;
  int nbricks, per_xcd;
  Box b;              // static dimensions; offset and velocity come from clk
  const Clock *clk;
  double rho0, omega;
  double om_ghost, om_bulk;  // multi-eigenvalue collision: -lambda_g, -lambda_v
  double kax, kdg;  // -6 w_q rho0 of the axis and of the diagonal directions
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

// Slot of sphere p in a brick's LDS table, or -1 if it is not there.
__device__ inline int table_find(const int32_t *skey, int p) {
  int h = p & (TSLOT - 1);
  for (int probe = 0; probe < TSLOT; ++probe) {
    const int key = skey[h];
    if (key == p) return h;
    if (key == -1) return -1;
    h = (h + 1) & (TSLOT - 1);
  }
  return -1;
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
};
template <> struct RowIO<float> {
  __device__ static float ld(__amdgpu_buffer_rsrc_t r, uint32_t off, int, H16) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  }
  __device__ static void st(__amdgpu_buffer_rsrc_t r, uint32_t off, float v, int, H16) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 0);
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

// Wait here for every outstanding vector-memory access (s_waitcnt vmcnt(0); expcnt and
// lgkmcnt left free), so that a rare branch that loads settles inside the branch instead
// of leaving the wait to the code after it, where it would hold up the common path.
__device__ inline void vm_settle() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Work-group barrier that orders LDS only: the lattice kernel's global stores are never
// read back within the kernel, so waiting for them at every z step would only add latency.
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// A wave-uniform value the compiler must treat as unknown at this point: row pointers built
// from it are formed where they are used, instead of being hoisted out of the loops into
// dozens of live scalar registers.
__device__ inline int opaque_uniform(int v) {
  v = __builtin_amdgcn_readfirstlane(v);
  asm volatile("" : "+s"(v));
  return v;
}
template <class T> __device__ inline T *opaque_uniform(T *p) {
  const uint64_t u = (uint64_t)p;
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u), hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  asm volatile("" : "+s"(lo), "+s"(hi));
  return (T *)(((uint64_t)hi << 32) | lo);
}

// One thread's view of its brick: the lane's column, the staged entries of the owner ring.
// A lane past the box end (xin false) computes a copy of the box's last column.
struct BrickView {
  int brick, t, lane, wv;
  int x0, z_lo, z_hi, y_lo, y_hi;
  bool xin;
  uint32_t xc, xm, xp;  // x of the node and of the pull sources c_x = +1, -1 (periodic)
};

// Brick of this work-group (XCD-aware order: hardware blocks are dealt round-robin to the 8
// XCDs; each XCD gets a contiguous range of bricks, z-major, so neighbouring bricks share
// its L2).  False for the surplus blocks of the last round.
__device__ inline bool brick_view(const LbmArgs &A, BrickView &V) {
  V.brick = (blockIdx.x & 7) * A.per_xcd + (blockIdx.x >> 3);
  if (V.brick >= A.nbricks) return false;
  const int bxi = V.brick % A.bxn;
  const int byi = (V.brick / A.bxn) % A.byn;
  const int bzi = V.brick / (A.bxn * A.byn);
  V.t = threadIdx.x;
  V.lane = V.t & 63;
  V.wv = __builtin_amdgcn_readfirstlane(V.t >> 6);
  V.x0 = bxi * TX;
  V.xin = V.x0 + V.lane < A.lx;
  V.xc = V.xin ? V.x0 + V.lane : A.lx - 1;
  V.xm = V.xc == 0 ? A.lx - 1 : V.xc - 1;
  V.xp = V.xc == (uint32_t)(A.lx - 1) ? 0 : V.xc + 1;
  V.z_lo = bzi * A.BZ;
  V.z_hi = min(A.lz, V.z_lo + A.BZ);
  V.y_lo = byi * A.BY;
  V.y_hi = min(A.ly, V.y_lo + A.BY);
  return true;
}

// Walk the brick.  For every row band: band(y, z_lo, sm, s0, sp, cen) once, with the staged
// owner planes z_lo-1, z_lo, z_lo+1; then for every z step node(par, y, live, z, sm, s0, sp,
// spp, cen, last, put) in every wave, with the staged planes z-1 .. z+2, the lane's centre
// entry and whether z is the band's last step; put() stores the plane fetched in this step
// into the ring (any time in the step: the slot it overwrites is no longer read).  par is
// Parity<0> on the band's even steps and Parity<1> on the odd ones.  A wave whose row lies
// past the box (the last band of a box whose ly is not a multiple of TY) walks a copy of
// row ly - 1, and a lane past the box end a copy of column lx - 1: live is false for them.
// The planes sit in a ring of NRING slots; each step fetches plane z+3.
constexpr int NRING = 5;
template <int P> struct Parity { static constexpr int v = P; };
template <class Band, class Fn>
__device__ inline void walk_brick(const LbmArgs &A, const BrickView &V, int32_t (*smap)[SPLANE],
                                  Band &&band, Fn &&node) {
  const int lx = A.lx, ly = A.ly, lz = A.lz, t = V.t;
  // the staged entries (row, column of a staged plane) of this thread: t and t + 256
  const bool two = t + 256 < SPLANE;
  const int e1 = two ? t + 256 : t;
  const int x0 = V.x0;
  int gx0 = (x0 - 1 + t % SROW) % lx, gx1 = (x0 - 1 + e1 % SROW) % lx;
  gx0 += gx0 < 0 ? lx : 0;
  gx1 += gx1 < 0 ? lx : 0;
  const int col = (int)V.xc - x0 + 1;  // the lane's column in a staged row
  for (int y0 = V.y_lo; y0 < V.y_hi; y0 += TY) {
    // source of each staged entry: a row of the owner map, or a ghost owner plane beyond
    // y = -1 and y = ly (rows past ly only feed copies)
    const int gy0 = y0 - 1 + t / SROW, gy1 = y0 - 1 + e1 / SROW;
    const int32_t *ep0 = gy0 < 0 ? A.gown + gx0
                       : gy0 >= ly ? A.gown + (size_t)lz * lx + gx0
                                   : A.own + gx0 + (size_t)lx * gy0;
    const int32_t *ep1 = gy1 < 0 ? A.gown + gx1
                       : gy1 >= ly ? A.gown + (size_t)lz * lx + gx1
                                   : A.own + gx1 + (size_t)lx * gy1;
    const int es0 = (gy0 < 0 || gy0 >= ly) ? lx : lx * ly;
    const int es1 = (gy1 < 0 || gy1 >= ly) ? lx : lx * ly;
    auto fetch = [&](int zz, int32_t &v0, int32_t &v1) {
      zz = zz < 0 ? zz + lz : (zz >= lz ? zz - lz : zz);  // zz in [-1, lz + 2], lz >= 8
      v0 = ep0[zz * es0];
      v1 = ep1[zz * es1];
    };
    {
      int32_t a0, a1, b0, b1, c0, c1, d0, d1;
      fetch(V.z_lo - 1, a0, a1);
      fetch(V.z_lo, b0, b1);
      fetch(V.z_lo + 1, c0, c1);
      fetch(V.z_lo + 2, d0, d1);
      __syncthreads();  // the previous row band is done with the ring
      smap[0][t] = a0; smap[1][t] = b0; smap[2][t] = c0; smap[3][t] = d0;
      if (two) { smap[0][e1] = a1; smap[1][e1] = b1; smap[2][e1] = c1; smap[3][e1] = d1; }
    }
    const bool rowlive = y0 + V.wv < ly;                 // uniform
    const int yb = rowlive ? y0 + V.wv : ly - 1;         // this wave's row (uniform)
    const bool live = rowlive && V.xin;
    const int cen = (yb - y0 + 1) * SROW + col;
    lds_barrier();  // the band's first planes are staged
    band(yb, V.z_lo, smap[0], smap[1], smap[2], cen);
    int r = 1;  // ring slot of plane zb
    auto step = [&](auto par, int zb) __attribute__((always_inline)) {
      lds_barrier();  // plane z+2 is staged; the slot of plane z-2 is free
      const int rm = r == 0 ? NRING - 1 : r - 1;
      const int rp = r == NRING - 1 ? 0 : r + 1;
      const int rpp = rp == NRING - 1 ? 0 : rp + 1;
      const int rw = rpp == NRING - 1 ? 0 : rpp + 1;  // = slot of plane z-2
      // plane z+3 for the step after next (past the brick's end it is fetched but unused)
      int32_t f0, f1;
      fetch(zb + 3, f0, f1);
      auto put = [&]() __attribute__((always_inline)) {
        smap[rw][t] = f0;
        if (two) smap[rw][e1] = f1;
      };
      node(par, yb, live, zb, smap[rm], smap[r], smap[rp], smap[rpp], cen, zb + 1 == V.z_hi, put);
      r = rp;
    };
    // two steps per trip (even and odd parity), so that a node can keep two register
    // sets without copying one into the other
    for (int zb = V.z_lo; zb < V.z_hi; zb += 2) {
      step(Parity<0>(), zb);
      if (zb + 1 < V.z_hi) step(Parity<1>(), zb + 1);
      else vm_settle();  // (an odd band length: keep the pending history of the loop)
    }
  }
}

// Owner of the source X - c_q of direction q, from the staged planes z-1, z, z+1.
__device__ inline int src_owner(int q, const int32_t *sm, const int32_t *s0, const int32_t *sp, int cen) {
  const int32_t *spl = cz(q) == 1 ? sm : (cz(q) == -1 ? sp : s0);
  return spl[cen - cy(q) * SROW - cx(q)];
}

// The node's links: bit q of the result is set if the source X - c_q is solid; *ph = the
// largest owner among them (-1 if none).
__device__ inline uint32_t link_bits(const int32_t *sm, const int32_t *s0, const int32_t *sp, int cen, int *ph) {
  uint32_t all = 0;
  int h = -1;
#pragma unroll
  for (int q = 1; q < NQ; ++q) {
    const int o = src_owner(q, sm, s0, sp, cen);
    all |= o >= 0 ? 1u << q : 0u;
    h = max(h, o);
  }
  *ph = h;
  return all;
}

// Spheres linked to a node, visited in descending id order; fn(p, m) handles sphere p
// whose links are the bits of m.  False if links were left over (more than six spheres).
template <class Fn>
__device__ inline bool for_each_sphere(const int32_t *sm, const int32_t *s0, const int32_t *sp, int cen,
                                       uint32_t all, int ph, Fn &&fn) {
  uint32_t rem = all;
  int p = ph;
  for (int it = 0; rem != 0 && it < 6; ++it) {
    uint32_t m = 0;
    int nx = -1;
#pragma unroll
    for (int q = 1; q < NQ; ++q) {
      const int o = src_owner(q, sm, s0, sp, cen);
      if (o == p) m |= 1u << q;
      else if ((rem >> q) & 1u) nx = max(nx, o);
    }
    fn(p, m);
    rem &= ~m;
    p = nx;
  }
  return rem == 0;
}

// Number of set bits of m below this lane; position of the r-th (from 0) set bit of m.
__device__ inline int lane_rank(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ inline int nth_bit(uint64_t m, int r) {
  int pos = 0;
  const int c = __builtin_popcount((uint32_t)m);
  if (r >= c) { r -= c; m >>= 32; pos = 32; }
  uint32_t v = (uint32_t)m;
#pragma unroll
  for (int w = 16; w >= 1; w >>= 1) {
    const int c2 = __builtin_popcount(v & ((1u << w) - 1u));
    if (r >= c2) { r -= c2; v >>= w; pos += w; }
  }
  return pos;
}
// The value v of lane src (a 32-bit lane permute through LDS hardware; no LDS storage).
__device__ inline int lane_pull(int v, int src) { return __builtin_amdgcn_ds_bpermute(src << 2, v); }
__device__ inline float lane_pull(float v, int src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(src << 2, __builtin_bit_cast(int, v)));
}
__device__ inline double lane_pull(double v, int src) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)u);
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Directions q whose component k (0 x, 1 y, 2 z) of c_q equals sgn, as a bit mask.
__host__ __device__ constexpr uint32_t dir_mask(int k, int sgn) {
  uint32_t m = 0;
  for (int q = 1; q < NQ; ++q)
    if ((k == 0 ? cx(q) : k == 1 ? cy(q) : cz(q)) == sgn) m |= 1u << q;
  return m;
}

// The solid end X - c_q of every link in m lies in the image of the sphere nearest to X
// (D = X - R in that image) when each component of D - c_q stays inside the half period
// (with a small margin, so that no rounding can tip the choice); then the lever of each
// link is D - c_q / 2 and one minimum image serves all of them.  Fails only for nodes
// about half a period from the centre whose links point across it (thin boxes).
__device__ inline bool same_image(const Box &b, double Dx, double Dy, double Dz, uint32_t m) {
  constexpr double e = 1e-6;
  const double hx = 0.5 * b.Lx - e, hy = 0.5 * b.Ly - e, hz = 0.5 * b.Lz - e;
  bool ok = true;
  if (m & dir_mask(0, 1)) ok = ok && Dx - 1.0 >= -hx;
  if (m & dir_mask(0, -1)) ok = ok && Dx + 1.0 <= hx;
  if (m & dir_mask(1, 1)) ok = ok && Dy - 1.0 >= -hy;
  if (m & dir_mask(1, -1)) ok = ok && Dy + 1.0 <= hy;
  if (m & dir_mask(2, 1)) ok = ok && Dz - 1.0 >= -hz;
  if (m & dir_mask(2, -1)) ok = ok && Dz + 1.0 <= hz;
  return ok && fabs(Dx) <= hx && fabs(Dy) <= hy && fabs(Dz) <= hz;
}

// ---- k_lbm: pull (eq. 3), bounce-back on moving spheres (eq. 7) with the link sums
//      (eqs. 6, 9, 10), BGK collision (eq. 4) on the deviations, non-equilibrium momentum
//      flux per brick ----
//
// Memory pipeline.  Vector-memory waits count in issue order, so a wait for one load also
// waits for every load and store issued before it, and a load or store skipped by a branch
// leaves the compiler unsure of the count (it then waits for more).  Hence the hot path has
// no branch around a global access: lanes past the box end and waves past the last row
// compute a copy of the last column or row and store the same values to the same places,
// and each step issues, in this order, the owner plane z+3, the populations of the next
// node (link directions load the node's own opposite population instead of the pull), and
// this node's stores.  The spheres' states come from LDS.  A node therefore waits only for
// loads issued one step earlier.
// COLL 0: BGK; 1: the linearised operator with separate eigenvalues for the traceless
// stress (-1/tau), its trace (-1/tau_bulk) and the ghost modes (-1/tau_ghost).
template <class ST, int COLL>
__global__ __launch_bounds__(256, 2) void k_lbm(LbmArgs A) {
  using CT = typename Store<ST>::CT;
  __shared__ int32_t smap[NRING][SPLANE];
  __shared__ int32_t skey[TSLOT];
  // 4-byte arithmetic: sphere states in LDS, FP32 stress partials; FP64: states read from
  // memory, FP64 partials (the LDS budget of two work-groups per compute unit)
  constexpr bool PF = sizeof(CT) == 4;
  constexpr bool DEFER = std::is_same<ST, __half>::value;  // FP16 storage: convert at use
  using PT = typename std::conditional<PF, float, double>::type;
  __shared__ double sdat[PF ? TSLOT : 1][SDAT];  // R, U, W of each table entry
  __shared__ double sval[4][TSLOT][HYD];  // one copy per wave: a fixed summation order
  __shared__ PT spn[6][256];                // per-thread fluid stress partials
  BrickView V;
  if (!brick_view(A, V)) return;  // the whole work-group
  const Box bx = clock_box(A.b, A.clk, 0);
  const int t = V.t, lane = V.lane;
  const int lx = A.lx, ly = A.ly, lz = A.lz;
  const size_t plane = A.plane;
  // ---- the brick's table: the spheres listed for it, with their states ----
  for (int i = t; i < TSLOT; i += 256) skey[i] = -1;
  for (int i = t; i < 4 * TSLOT * HYD; i += 256) (&sval[0][0][0])[i] = 0.0;
#pragma unroll
  for (int c = 0; c < 6; ++c) spn[c][t] = (PT)0;
  __syncthreads();
  {
    const int cnt = min(A.bt_cnt[V.brick], TSLOT);  // past TSLOT: the global fallback
    for (int i = t; i < cnt; i += 256) table_slot(skey, A.bt_key[(size_t)V.brick * TSLOT + i]);
  }
  __syncthreads();
  for (int i = t; PF && i < TSLOT * 9; i += 256) {
    const int slot = i / 9, c = i - 9 * (i / 9);
    const int key = skey[slot];
    if (key >= 0) {
      const double *src = c < 3 ? A.R : (c < 6 ? A.U : A.W);
      sdat[slot][c] = src[3 * key + c % 3];
    }
  }
  // (the first row band's barrier orders these writes before any use)
  const CT om = (CT)A.omega;
  const CT rho0 = (CT)A.rho0;
  constexpr uint32_t es = sizeof(ST), ges = sizeof(CT);
  const __amdgpu_buffer_rsrc_t rin = buf_rsrc(A.fin, A.pop_bytes), rout = buf_rsrc(A.fout, A.pop_bytes);
  const __amdgpu_buffer_rsrc_t rgh = buf_rsrc(A.gval, A.gval_bytes);
  // byte offsets of the lane's column and of its pull sources c_x = +1, -1
  const uint32_t xcb = V.xc * es, xmb = V.xm * es, xpb = V.xp * es;
  const uint32_t xcg = V.xc * ges, xmg = V.xm * ges, xpg = V.xp * ges;
  // The populations a node needs: for a link direction q (bit q of lk: X - c_q is solid)
  // the node's own opposite population n*_qbar(X), which bounce-back sends back (eq. 7),
  // else the pull source n*_q(X - c_q) (eq. 3).  Every lane loads (a solid node's values
  // are replaced by the rest state).
  auto load_node = [&](int yb, int zb, uint32_t lk, CT *dst) __attribute__((always_inline)) {
    const int y = opaque_uniform(yb), z = opaque_uniform(zb);
    const uint32_t pb = (uint32_t)opaque_uniform((int)(plane * es));  // plane stride, bytes
    const int zm = z == 0 ? lz - 1 : z - 1, zp = z == lz - 1 ? 0 : z + 1;
    const uint32_t rowc = (uint32_t)((z * ly + y) * lx) * es;  // byte offset of the row in a plane
    if constexpr (DEFER) dst[0] = RowIO<ST>::raw(rin, rowc + xcb);
    else dst[0] = RowIO<ST>::ld(rin, rowc + xcb, 0, A.h16);
    // one load per direction, no branch (a pull across a sliding plane reads some row of
    // the array, or nothing, and is replaced below)
#pragma unroll
    for (int q = 1; q < NQ; ++q) {
      const bool lq = (lk >> q) & 1u;
      const uint32_t own_off = opp(q) * pb + rowc + xcb;  // w_qbar = w_q: same FP16 scale
      const int ys = y - cy(q);
      const int zs = cz(q) == 1 ? zm : (cz(q) == -1 ? zp : z);
      const uint32_t xsb = cx(q) == 1 ? xmb : (cx(q) == -1 ? xpb : xcb);
      const uint32_t pull_off = q * pb + (uint32_t)((zs * ly + ys) * lx) * es + xsb;
      if constexpr (DEFER) dst[q] = RowIO<ST>::raw(rin, lq ? own_off : pull_off);
      else dst[q] = RowIO<ST>::ld(rin, lq ? own_off : pull_off, q, A.h16);
    }
    if (y == 0 || y == ly - 1) {  // uniform: directions across the sliding plane read the
                                  // Lees-Edwards ghost row (these rows do not overlap)
      const int side = y == 0 ? 0 : 1;
      CT g[5];
#pragma unroll
      for (int q = 1; q < NQ; ++q) {
        if (cy(q) == (side == 0 ? 1 : -1)) {
          const int zs = cz(q) == 1 ? zm : (cz(q) == -1 ? zp : z);
          const uint32_t xsg = cx(q) == 1 ? xmg : (cx(q) == -1 ? xpg : xcg);
          g[gslot(q)] = RowIO<CT>::ld(rgh, (uint32_t)(((side * 5 + gslot(q)) * lz + zs) * lx) * ges + xsg, q, A.h16);
        }
      }
      vm_settle();
      if constexpr (DEFER) {  // an edge row's node is converted here, whole
#pragma unroll
        for (int q = 0; q < NQ; ++q) dst[q] = RowIO<ST>::dec(dst[q], q, A.h16);
      }
#pragma unroll
      for (int q = 1; q < NQ; ++q) {
        if (cy(q) == (side == 0 ? 1 : -1)) {
          const bool lq = (lk >> q) & 1u;
          dst[q] = lq ? dst[q] : g[gslot(q)];
        }
      }
    }
  };
  // With 4-byte arithmetic a step loads the next node while it computes (two register sets:
  // even steps work on ra and load into rb, odd steps the other way round); in FP64 each
  // node loads its own (register budget).
  CT ra[NQ], rb[NQ];
  bool nfl = false;      // the next node is a fluid node
  uint32_t nall = 0;     // its link directions
  int nph = -1;          // the largest sphere id among them
#pragma unroll
  for (int q = 0; q < NQ; ++q) { ra[q] = 0; rb[q] = 0; }
  // n: this node's populations in, post-collision populations out (0 = rest state if
  // solid); pn: the next node's loads.  live: the lane's node is its own (not a copy).
  auto node = [&](CT (&n)[NQ], CT (&pn)[NQ], int yb, bool live, int zb, const int32_t *sm,
                  const int32_t *s0, const int32_t *sp, const int32_t *spp, int cen, bool last,
                  auto &&put) __attribute__((always_inline)) {
    const int y = opaque_uniform(yb), z = opaque_uniform(zb);
    const uint32_t pb = (uint32_t)opaque_uniform((int)(plane * es));  // plane stride, bytes
    const uint32_t rowc = (uint32_t)((z * ly + y) * lx) * es;  // byte offset of the row in a plane
    bool fl;           // fluid node
    uint32_t all = 0;  // its link directions (bit q: X - c_q is solid)
    int ph = -1;       // the largest sphere id among them
    if (PF) {
      fl = nfl; all = nall; ph = nph;
    } else {
      fl = s0[cen] == -1;
      if (fl) all = link_bits(sm, s0, sp, cen, &ph);
      load_node(yb, zb, all, n);
    }
    if (PF && !last) {
      nfl = sp[cen] == -1;
      nall = 0;
      nph = -1;
      if (nfl) nall = link_bits(s0, sp, spp, cen, &nph);
      load_node(yb, zb + 1, nall, pn);
    } else if (PF) {
      vm_settle();  // a band's last step: nothing to overlap
#pragma unroll
      for (int q = 0; q < NQ; ++q) pn[q] = 0;  // (the old values are dead on every path)
    }
    if constexpr (DEFER) {  // the stored 16 bits to values (edge rows: done at the load)
      if (fl && !(y == 0 || y == ly - 1)) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) n[q] = RowIO<ST>::dec(n[q], q, A.h16);
      }
    }
    // bounce-back and link sums of sphere p over the links m of the node in column x (the
    // lane's own node, or, for a helper lane, the node it was handed); live: the node is
    // not a copy, so its sums count
    auto body = [&](int p, uint32_t m, int x, bool live) __attribute__((always_inline)) {
        // the sphere's state: from the brick's table, else (not listed) from memory
        const int slot = table_find(skey, p);
        double Rx, Ry, Rz, U0, U1, U2, w0, w1, w2;
        if (PF) {
          const int sl = slot >= 0 ? slot : 0;
          Rx = sdat[sl][0]; Ry = sdat[sl][1]; Rz = sdat[sl][2];
          U0 = sdat[sl][3]; U1 = sdat[sl][4]; U2 = sdat[sl][5];
          w0 = sdat[sl][6]; w1 = sdat[sl][7]; w2 = sdat[sl][8];
          if (slot < 0) {  // rare: not listed (full table)
            Rx = A.R[3 * p]; Ry = A.R[3 * p + 1]; Rz = A.R[3 * p + 2];
            U0 = A.U[3 * p]; U1 = A.U[3 * p + 1]; U2 = A.U[3 * p + 2];
            w0 = A.W[3 * p]; w1 = A.W[3 * p + 1]; w2 = A.W[3 * p + 2];
            vm_settle();
          }
        } else {
          Rx = A.R[3 * p]; Ry = A.R[3 * p + 1]; Rz = A.R[3 * p + 2];
          U0 = A.U[3 * p]; U1 = A.U[3 * p + 1]; U2 = A.U[3 * p + 2];
          w0 = A.W[3 * p]; w1 = A.W[3 * p + 1]; w2 = A.W[3 * p + 2];
        }
        double Dx, Dy, Dz;
        int k;
        minimage(bx, (double)x - Rx, (double)y - Ry, (double)z - Rz, Dx, Dy, Dz, k);
        double v[HYD];
        if (same_image(bx, Dx, Dy, Dz, m)) {
          // rigid-body velocity at the node (eq. 8)
          const double ux = U0 + k * bx.ule + (w1 * Dz - w2 * Dy);
          const double uy = U1 + (w2 * Dx - w0 * Dz);
          const double uz = U2 + (w0 * Dy - w1 * Dx);
          double g0 = 0, g1 = 0, g2 = 0, mxx = 0, myy = 0, mzz = 0, mxy = 0, mxz = 0, myz = 0;
#pragma unroll
          for (int pi = 0; pi < 9; ++pi) {
            const int q = 2 * pi + 1, b = q + 1;
            const double corr = (q <= 6 ? A.kax : A.kdg) * cdot<double>(q, ux, uy, uz);
            const bool lq = (m >> q) & 1u, lb = (m >> b) & 1u;
            const double fq = (double)n[q], fb = (double)n[b];
            const double mq = lq ? fma(2.0, fq, -corr) : 0.0;
            const double mb = lb ? fma(2.0, fb, corr) : 0.0;
            const double sm2 = mq + mb, df = mq - mb;
            // each sum starts at its first contributing pair (no addition to zero)
            acc_pair(g0, pi, 0, cx(q), df); acc_pair(g1, pi, 1, cy(q), df); acc_pair(g2, pi, 2, cz(q), df);
            acc_pair(mxx, pi, 0, cx(q) * cx(q), sm2);
            acc_pair(myy, pi, 1, cy(q) * cy(q), sm2);
            acc_pair(mzz, pi, 2, cz(q) * cz(q), sm2);
            acc_pair(mxy, pi, 3, cx(q) * cy(q), sm2); acc_pair(mxz, pi, 4, cx(q) * cz(q), sm2);
            acc_pair(myz, pi, 5, cy(q) * cz(q), sm2);
            const CT cr = (CT)corr;
            if (lq) n[q] = n[q] - cr;
            if (lb) n[b] = n[b] + cr;
          }
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
        } else {
          // rare: each link with the lever of the image that holds its solid end (eq. 8)
#pragma unroll
          for (int c = 0; c < 12; ++c) v[c] = 0.0;
#pragma unroll
          for (int q = 1; q < NQ; ++q) {
            if ((m >> q) & 1u) {
              double ex, ey, ez;
              int kq;
              minimage(bx, (double)(x - cx(q)) - Rx, (double)(y - cy(q)) - Ry, (double)(z - cz(q)) - Rz,
                       ex, ey, ez, kq);
              const double lvx = ex + 0.5 * cx(q), lvy = ey + 0.5 * cy(q), lvz = ez + 0.5 * cz(q);
              const double ubx = U0 + kq * bx.ule + (w1 * lvz - w2 * lvy);
              const double uby = U1 + (w2 * lvx - w0 * lvz);
              const double ubz = U2 + (w0 * lvy - w1 * lvx);
              const double corr = (q <= 6 ? A.kax : A.kdg) * cdot<double>(q, ubx, uby, ubz);
              const double fo = (double)n[q];
              n[q] = (CT)(fo - corr);
              const double mm = fma(2.0, fo, -corr);
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
          }
        }
        v[12] = (double)__builtin_popcount(m);
        if (live) {
          if (slot >= 0) {  // LDS atomics (the two address spaces kept apart: no flat atomics)
#pragma unroll
            for (int c = 0; c < HYD; ++c) unsafeAtomicAdd(&sval[V.wv][slot][c], v[c]);
          } else {
#pragma unroll
            for (int c = 0; c < HYD; ++c) unsafeAtomicAdd(&A.hyd_fb[(size_t)p * HYD + c], v[c]);
          }
        }
    };
    if constexpr (PF) {
      // The node's first sphere (ph) and second sphere (p2) with their links m1, m2.  Nearly
      // every row has some node between two spheres, and a second pass over the links
      // would cost the whole wave a pass; instead each second sphere is handed to a lane of
      // the wave whose own node is solid (its registers are free): it takes the node's
      // populations, runs the same pass beside the first spheres and hands the corrected
      // ones back.  Third spheres, and second spheres left over when the wave has too few
      // solid nodes, take further passes.  The assignment depends only on the row's
      // geometry, so the sums stay bitwise reproducible.
      uint32_t m1 = 0, m2 = 0;
      int p2 = -1;
      if (fl && all) {
#pragma unroll
        for (int q = 1; q < NQ; ++q) {
          const int o = src_owner(q, sm, s0, sp, cen);
          if (o == ph) m1 |= 1u << q;
          else if (o >= 0) p2 = max(p2, o);
        }
        if (p2 >= 0) {
#pragma unroll
          for (int q = 1; q < NQ; ++q) m2 |= src_owner(q, sm, s0, sp, cen) == p2 ? 1u << q : 0u;
        }
      }
      const bool needs = p2 >= 0;
      const uint64_t needm = __builtin_amdgcn_ballot_w64(needs), helpm = __builtin_amdgcn_ballot_w64(!fl);
      const int nneed = __builtin_popcountll(needm), nhelp = __builtin_popcountll(helpm);
      const int rneed = lane_rank(needm), rhelp = lane_rank(helpm);
      const bool task = !fl && rhelp < nneed;       // a solid lane with a handed-over node
      const bool handed = needs && rneed < nhelp;   // a node whose second sphere was handed over
      const int src = task ? nth_bit(needm, rhelp) : lane;
      const int hlp = handed ? nth_bit(helpm, rneed) : lane;
      const int tp = lane_pull(p2, src), tx = lane_pull((int)V.xc, src), tl = lane_pull((int)live, src);
      const uint32_t tm = (uint32_t)lane_pull((int)m2, src);
#pragma unroll
      for (int q = 1; q < NQ; ++q) {
        const CT v = lane_pull(n[q], src);
        n[q] = task ? v : n[q];
      }
      int pp = fl ? ph : (task ? tp : -1);
      uint32_t mm = fl ? m1 : tm;
      int xx = fl ? (int)V.xc : tx;
      bool lv = fl ? live : (task && tl != 0);
      uint32_t lrem = fl ? (all & ~m1 & ~(handed ? m2 : 0u)) : 0u;  // links of later passes
      for (int it = 0; it < 6; ++it) {
        if (it > 0) {  // the next sphere among the remaining links (largest id first)
          int pnx = -1;
#pragma unroll
          for (int q = 1; q < NQ; ++q) {
            const int o = src_owner(q, sm, s0, sp, cen);
            pnx = (lrem >> q) & 1u ? max(pnx, o) : pnx;
          }
          uint32_t mn = 0;
#pragma unroll
          for (int q = 1; q < NQ; ++q) mn |= ((lrem >> q) & 1u) && src_owner(q, sm, s0, sp, cen) == pnx ? 1u << q : 0u;
          pp = lrem ? pnx : -1;
          mm = mn;
          xx = (int)V.xc;
          lv = live;
          lrem &= ~mn;
        }
        if (pp >= 0 && mm) body(pp, mm, xx, lv);
        if (it == 0) {  // the handed-over nodes' corrected populations go back
#pragma unroll
          for (int q = 1; q < NQ; ++q) {
            const CT v = lane_pull(n[q], hlp);
            n[q] = handed && ((m2 >> q) & 1u) ? v : n[q];
          }
        }
        if (__builtin_amdgcn_ballot_w64(lrem != 0) == 0) break;
      }
      if (lrem != 0 && live) atomicOr(A.flags, 8);
    }
    if (fl) {
      if constexpr (!PF) {
        const bool done = for_each_sphere(sm, s0, sp, cen, all, ph,
                                          [&](int p, uint32_t m) { body(p, m, (int)V.xc, live); });
        if (!done && live) atomicOr(A.flags, 8);
      }
      // ---- moments and BGK collision on the deviations d_q = n_q - w_q rho0, opposite
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
      const CT ir = (CT)1 / rho;
      const CT ux = jx * ir, uy = jy * ir, uz = jz * ir;
      const CT uu = ux * ux + uy * uy + uz * uz;
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
      // non-equilibrium momentum flux Pi^neq = sum_q (n_q - feq_q) c_q c_q (pairs add)
      CT s[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int pi = 0; pi < 9; ++pi) {
        const int q = 2 * pi + 1;
        if (cx(q) != 0) s[0] += ps[pi];
        if (cy(q) != 0) s[1] += ps[pi];
        if (cz(q) != 0) s[2] += ps[pi];
        addc(s[3], cx(q) * cy(q), ps[pi]);
        addc(s[4], cx(q) * cz(q), ps[pi]);
        addc(s[5], cy(q) * cz(q), ps[pi]);
      }
      if (live) {
#pragma unroll
        for (int c = 0; c < 6; ++c) spn[c][t] += (PT)s[c];
      }
    } else {
#pragma unroll
      for (int q = 0; q < NQ; ++q) n[q] = 0;
    }
    put();  // the owner plane fetched this step, into the ring
    // every node of the row is stored, so that the wave writes whole cache lines (HBM3E
    // has no write mask: a partly written line costs a read-modify-write); copies store
    // what the node's own lane or wave stores
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      RowIO<ST>::st(rout, q * pb + rowc + xcb, n[q], q, A.h16);
  };
  walk_brick(A, V, smap,
             [&](int yb, int z_lo, const int32_t *sm, const int32_t *s0, const int32_t *sp, int cen) {
    if (!PF) return;
    nfl = s0[cen] == -1;
    nall = 0;
    nph = -1;
    if (nfl) nall = link_bits(sm, s0, sp, cen, &nph);
    load_node(yb, z_lo, nall, ra);
    vm_settle();  // once per band: the steps then see one history of pending accesses
  }, [&](auto par, int yb, bool live, int zb, const int32_t *sm, const int32_t *s0, const int32_t *sp,
         const int32_t *spp, int cen, bool last, auto &&put) {
    if constexpr (decltype(par)::v == 0) node(ra, rb, yb, live, zb, sm, s0, sp, spp, cen, last, put);
    else node(rb, ra, yb, live, zb, sm, s0, sp, spp, cen, last, put);
  });
  __syncthreads();
  // ---- brick table out ----
  for (int i = t; i < TSLOT; i += 256) {
    const int key = skey[i];
    A.bt_key[(size_t)V.brick * TSLOT + i] = key;
    if (key >= 0) {
      for (int c = 0; c < HYD; ++c)
        A.bt_val[((size_t)V.brick * TSLOT + i) * HYD + c] = ((sval[0][i][c] + sval[1][i][c]) + sval[2][i][c]) + sval[3][i][c];
      // entries with links go on the sphere's list (k_hydro_gather orders them by index)
      const double nl = ((sval[0][i][HYD - 1] + sval[1][i][HYD - 1]) + sval[2][i][HYD - 1]) + sval[3][i][HYD - 1];
      if (nl > 0.0) {
        const int c = atomicAdd(&A.sp_cnt[key], 1);
        if (c < SPCAP) A.sp_ent[(size_t)key * SPCAP + c] = V.brick * TSLOT + i;
      }
    }
  }
  // ---- brick partial of the non-equilibrium momentum flux (fluid stress): the 256
  //      per-thread partials of each component summed by one wave in a fixed order ----
  if (V.wv == 0) {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double v = wave_sum(((double)spn[c][lane] + (double)spn[c][lane + 64]) +
                                ((double)spn[c][lane + 128] + (double)spn[c][lane + 192]));
      if (lane == 0) A.pineq[(size_t)V.brick * 6 + c] = v;
    }
  }
}

static LbmArgs lbm_args(Sim *s, const Box &b) {
  LbmArgs A;
  A.fin = s->f[s->cur];
  A.fout = s->f[1 - s->cur];
  A.plane = s->plane;
  {
    const size_t es = s->precision == 0 ? 8 : s->precision == 1 ? 4 : 2;
    const size_t ges = s->precision == 0 ? 8 : 4;
    A.pop_bytes = (uint32_t)(NQ * s->plane * es);  // < 2^32, checked at creation
    A.gval_bytes = (uint32_t)(10 * (size_t)s->lx * s->lz * ges);
  }
  A.own = s->own;
  A.gown = s->gown;
  A.gval = s->gval;
  A.R = s->R[s->pcur];
  A.U = s->U[s->pcur];
  A.W = s->W[s->pcur];
  A.bt_key = s->bt_key;
  A.bt_cnt = s->bt_cnt;
  A.bt_val = s->bt_val;
  A.sp_cnt = s->sp_cnt;
  A.sp_ent = s->sp_ent;
  A.hyd_fb = s->hyd_fb;
  A.pineq = s->pineq;
  A.flags = s->flags;
  A.lx = s->lx; A.ly = s->ly; A.lz = s->lz;
  A.bxn = s->bxn; A.byn = s->byn; A.bzn = s->bzn; A.BY = s->BY; A.BZ = s->BZ;
  A.nbricks = s->nbricks;
  A.per_xcd = (s->nbricks + 7) / 8;
  A.b = b;
  A.clk = s->clk;
  A.rho0 = s->rho0;
  A.omega = 1.0 / s->tau;
  A.om_ghost = 1.0 / s->tau_ghost;
  A.om_bulk = 1.0 / s->tau_bulk;
  A.kax = -6.0 * wq(1) * s->rho0;
  A.kdg = -6.0 * wq(7) * s->rho0;
  A.h16 = s->h16;
  return A;
}

hipError_t launch_lbm(Sim *s, const Box &b) {
  const LbmArgs A = lbm_args(s, b);
  dim3 grid(A.per_xcd * 8), blk(256);
  if (s->collision == 0) {
    if (s->precision == 0) hipLaunchKernelGGL((k_lbm<double, 0>), grid, blk, 0, s->stream, A);
    else if (s->precision == 1) hipLaunchKernelGGL((k_lbm<float, 0>), grid, blk, 0, s->stream, A);
    else hipLaunchKernelGGL((k_lbm<__half, 0>), grid, blk, 0, s->stream, A);
  } else {
    if (s->precision == 0) hipLaunchKernelGGL((k_lbm<double, 1>), grid, blk, 0, s->stream, A);
    else if (s->precision == 1) hipLaunchKernelGGL((k_lbm<float, 1>), grid, blk, 0, s->stream, A);
    else hipLaunchKernelGGL((k_lbm<__half, 1>), grid, blk, 0, s->stream, A);
  }
  return hipGetLastError();
}

// Bricks near a sphere.  The lattice kernel's table for a brick must hold every sphere
// whose owner entries its staged region (the brick and a one-node halo, with the ghost
// rows beyond y = -1 and y = ly) can hold: nodes within a_map of one of the sphere's
// Lees-Edwards images (at R + k (s, Ly, 0)), hence every brick with a node within a_map + 2
// of an image.  The same enumeration lists the spheres for each brick (k_brick_lists) and
// gathers a sphere's sums (k_hydro_gather).
struct BrickGeo {
  int lx, ly, lz, bxn, byn, BY, BZ;
};

// Next node coordinate (along a periodic axis of length L with bricks of B nodes, the last
// one shorter when B does not divide L) that starts a new brick after coordinate xx.
__device__ inline int next_brick_start(int xx, int L, int B) {
  int w = xx % L;
  w = w < 0 ? w + L : w;
  const int nxt = (w / B + 1) * B;  // start of the following brick, or past the axis end
  return xx + ((nxt < L ? nxt : L) - w);
}
__device__ inline int brick_of(int xx, int L, int B) {
  int w = xx % L;
  w = w < 0 ? w + L : w;
  return w / B;
}

// fn(brick) for every brick with a node within r of an image of the sphere at Rp (LE offset
// s), each once, in a fixed order; run by a whole wave, fn in every lane.  vis: the wave's
// list of visited bricks (a wrapped range can reach a brick twice; past 256 entries a
// brick may be visited again).
template <class F>
__device__ inline void sphere_bricks(const BrickGeo &G, const double *Rp, double r, double s,
                                     int *vis, int lane, F &&fn) {
  // a runaway (or non-finite) position of a failed run: no bricks, and no loop whose bounds
  // come from a coordinate far outside the box
  if (!(Rp[0] > -2.0 * G.lx && Rp[0] < 3.0 * G.lx && Rp[1] > -2.0 * G.ly && Rp[1] < 3.0 * G.ly &&
        Rp[2] > -2.0 * G.lz && Rp[2] < 3.0 * G.lz && r < 0.5 * G.lx + 0.5 * G.ly + 0.5 * G.lz))
    return;
  int nvis = 0;
  int zlo = (int)floor(Rp[2] - r), zhi = (int)ceil(Rp[2] + r);
  if (zhi - zlo + 1 >= G.lz) { zlo = 0; zhi = G.lz - 1; }
  for (int k = -1; k <= 1; ++k) {
    const double cy_ = Rp[1] + k * (double)G.ly;
    int ylo = (int)floor(cy_ - r), yhi = (int)ceil(cy_ + r);
    if (ylo < 0) ylo = 0;
    if (yhi > G.ly - 1) yhi = G.ly - 1;
    if (ylo > yhi) continue;
    const double cx_ = Rp[0] + k * s;
    int xlo = (int)floor(cx_ - r), xhi = (int)ceil(cx_ + r);
    if (xhi - xlo + 1 >= G.lx) { xlo = 0; xhi = G.lx - 1; }
    for (int zz = zlo; zz <= zhi; zz = next_brick_start(zz, G.lz, G.BZ)) {
      const int bz = brick_of(zz, G.lz, G.BZ);
      for (int by = ylo / G.BY; by <= yhi / G.BY; ++by) {
        for (int xx = xlo; xx <= xhi; xx = next_brick_start(xx, G.lx, TX)) {
          const int brick = brick_of(xx, G.lx, TX) + G.bxn * (by + G.byn * bz);
          bool dup = false;
          for (int base = 0; base < nvis; base += 64) {
            const int v = base + lane < nvis ? vis[base + lane] : -1;
            if (__ballot(v == brick)) { dup = true; break; }
          }
          if (dup) continue;
          if (nvis < 256) {
            if (lane == 0) vis[nvis] = brick;
            ++nvis;
            __builtin_amdgcn_wave_barrier();
          }
          fn(brick);
        }
      }
    }
  }
}

// ---- k_brick_lists: each sphere appends its id to the list of every brick near it (one
//      wave per sphere; the list order is immaterial: the brick's sums are kept per sphere)
struct ListArgs {
  const double *R, *amap;
  int32_t *bt_key, *bt_cnt;
  int n;
  BrickGeo G;
  const Clock *clk;
};

__global__ __launch_bounds__(256) void k_brick_lists(ListArgs A) {
  __shared__ int vis[4][256];
  const int wv = threadIdx.x >> 6;
  const int p = blockIdx.x * 4 + wv;
  const int lane = threadIdx.x & 63;
  if (p >= A.n) return;  // uniform per wave
  if (!(isfinite(A.R[3 * p]) && isfinite(A.R[3 * p + 1]) && isfinite(A.R[3 * p + 2]))) return;
  // the enumeration keeps the first 256 distinct bricks in vis; their appends are issued by
  // the lanes together afterwards (a returning atomic per brick in turn would serialise)
  int ncall = 0;
  auto append = [&](int brick) {
    const int c = atomicAdd(&A.bt_cnt[brick], 1);
    if (c < TSLOT) A.bt_key[(size_t)brick * TSLOT + c] = p;
  };
  sphere_bricks(A.G, &A.R[3 * p], A.amap[p] + 2.0, A.clk->cur.s, vis[wv], lane, [&](int brick) {
    if (ncall >= 256 && lane == 0) append(brick);
    ++ncall;
  });
  __builtin_amdgcn_wave_barrier();
  const int m = ncall < 256 ? ncall : 256;
  for (int k = lane; k < m; k += 64) append(vis[wv][k]);
}

static BrickGeo brick_geo(const Sim *s) {
  BrickGeo G;
  G.lx = s->lx; G.ly = s->ly; G.lz = s->lz;
  G.bxn = s->bxn; G.byn = s->byn; G.BY = s->BY; G.BZ = s->BZ;
  return G;
}

hipError_t launch_brick_lists(Sim *s) {
  hipError_t e = launch_fill_i32(s->bt_cnt, (size_t)s->nbricks, 0, s->stream);
  if (e != hipSuccess || s->n == 0) return e;
  ListArgs A;
  A.R = s->R[s->pcur]; A.amap = s->amap;
  A.bt_key = s->bt_key; A.bt_cnt = s->bt_cnt;
  A.n = s->n;
  A.G = brick_geo(s);
  A.clk = s->clk;
  hipLaunchKernelGGL(k_brick_lists, dim3((s->n + 3) / 4), dim3(256), 0, s->stream, A);
  return hipGetLastError();
}

// Per-sphere hydrodynamic sums, one wave per sphere.  k_lbm lists each sphere's table
// entries with links (at most SPCAP); the wave sorts them by index (brick, then slot) so that
// the order does not depend on how the flushes interleaved, and adds them by a fixed lane
// butterfly.  A sphere with more entries (tiny bricks) visits every brick near it instead,
// in enumeration order.  Either way the overflow accumulator is added and cleared, and so is
// the entry count, for the next step.
struct GatherArgs {
  const double *R, *amap;
  const int32_t *bt_key;
  const double *bt_val;
  int32_t *sp_cnt;
  const int32_t *sp_ent;
  double *hyd_fb;
  double *hyd;
  int n;
  BrickGeo G;
  const Clock *clk;  // LE offset of the step
};

__global__ __launch_bounds__(256) void k_hydro_gather(GatherArgs A) {
  __shared__ int vis[4][256];
  const int wv = threadIdx.x >> 6;
  const int p = blockIdx.x * 4 + wv;
  const int lane = threadIdx.x & 63;
  if (p >= A.n) return;  // uniform per wave
  double acc[HYD], fb[HYD];
#pragma unroll
  for (int c = 0; c < HYD; ++c) acc[c] = 0.0;
  // the count, the entry slots (SPCAP per sphere, read whole) and the overflow accumulator are
  // independent loads, issued together
  const int cnt = A.sp_cnt[p];
  const int ent = A.sp_ent[(size_t)p * SPCAP + lane];
#pragma unroll
  for (int c = 0; c < HYD; ++c) fb[c] = lane == 0 ? A.hyd_fb[(size_t)p * HYD + c] : 0.0;
  if (cnt <= SPCAP) {
    // the entries, sorted ascending across the wave (bitonic; empty lanes sort last)
    int e = lane < cnt ? ent : 0x7fffffff;
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1) {
        const int o = __shfl_xor(e, j, 64);
        const bool up = (lane & k) == 0, low = (lane & j) == 0;
        e = (low == up) ? min(e, o) : max(e, o);
      }
    }
    double v[HYD];
#pragma unroll
    for (int c = 0; c < HYD; ++c) v[c] = lane < cnt ? A.bt_val[(size_t)e * HYD + c] : 0.0;
#pragma unroll
    for (int c = 0; c < HYD; ++c) acc[c] = wave_sum(v[c]);
  } else if (isfinite(A.R[3 * p]) && isfinite(A.R[3 * p + 1]) && isfinite(A.R[3 * p + 2])) {
    sphere_bricks(A.G, &A.R[3 * p], A.amap[p] + 2.0, A.clk->cur.s, vis[wv], lane, [&](int brick) {
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
    });
  }
  if (lane == 0) {
    for (int c = 0; c < HYD; ++c) {
      A.hyd[(size_t)p * HYD + c] = acc[c] + fb[c];
      A.hyd_fb[(size_t)p * HYD + c] = 0.0;
    }
    A.sp_cnt[p] = 0;
  }
}

hipError_t launch_hydro_gather(Sim *s, const Box &b) {
  GatherArgs A;
  A.R = s->R[s->pcur]; A.amap = s->amap;
  A.bt_key = s->bt_key; A.bt_val = s->bt_val; A.hyd_fb = s->hyd_fb;
  A.sp_cnt = s->sp_cnt; A.sp_ent = s->sp_ent;
  A.hyd = s->hyd[s->hcur];
  A.n = s->n;
  A.G = brick_geo(s);
  A.clk = s->clk;
  (void)b;
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
  Box b;             // with clk set, offset and velocity come from the clock
  const Clock *clk;
  int lx, ly, lz, n;
  double rho0;
  int values;
  int32_t *gown;
  void *gval;
  int32_t *flags;
  H16 h16;
  // with lists set: the spheres listed for each brick (k_brick_lists of this step), which
  // hold every sphere that can own a ghost point of the brick's first or last row band
  const int32_t *bt_key, *bt_cnt;
  int lists, bxn, byn, BZ;
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

// One thread per ghost point (x, z) of the two ghost planes: owner, then (fluid points) the
// values.  The spheres of the brick that holds the first lane's point are staged in LDS for
// the wave (every lane's brick when the row length is a multiple of the brick width); a lane
// in another brick reads its own list from memory, and a brick whose list overflowed falls
// back to the cell list.
template <class ST>
__global__ __launch_bounds__(256) void k_ghosts(GhostArgs A) {
  using CT = typename Store<ST>::CT;
  __shared__ double s_sph[4][TSLOT][4];
  __shared__ int32_t s_id[4][TSLOT];
  const Box bx = clock_box(A.b, A.clk, 0);
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int npl = A.lx * A.lz;
  const bool live = idx < 2 * npl;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int id = live ? idx : 2 * npl - 1;  // lanes past the end take the last point (no stores)
  const int g = id / npl;
  const int rem = id - g * npl;
  const int z = rem / A.lx, x = rem - (rem / A.lx) * A.lx;
  const double gy = g == 0 ? -1.0 : (double)A.ly;
  // primary-box position of the ghost point, for the cell search only
  double px = g == 0 ? (double)x + bx.s : (double)x - bx.s;
  px = px - bx.Lx * floor(px / bx.Lx);
  const double py = g == 0 ? (double)(A.ly - 1) : 0.0;
  int owner = -1, clash = 0;
  auto test = [&](int p, double Rx, double Ry, double Rz, double am) {
    double dx, dy2, dz;
    int k;
    minimage(bx, (double)x - Rx, gy - Ry, (double)z - Rz, dx, dy2, dz, k);
    const double r2 = dx * dx + dy2 * dy2 + dz * dz;
    if (r2 < am * am) {
      if (owner >= 0 && owner != p) clash = 1;
      if (owner < 0 || p < owner) owner = p;
    }
  };
  auto test_mem = [&](int p) { test(p, A.R[3 * p], A.R[3 * p + 1], A.R[3 * p + 2], A.amap[p]); };
  const bool use_lists = A.n > 0 && A.lists;
  const int brick = use_lists ? x / TX + A.bxn * ((g == 0 ? 0 : A.byn - 1) + A.byn * (z / A.BZ)) : 0;
  const int b0 = __shfl(brick, 0, 64);
  const int c0 = use_lists ? A.bt_cnt[b0] : 0;
  const bool staged = use_lists && c0 <= TSLOT;
  if (staged) {
    const int32_t *key = A.bt_key + (size_t)b0 * TSLOT;
    for (int i = lane; i < c0; i += 64) {
      const int p = key[i];
      s_id[wv][i] = p;
      s_sph[wv][i][0] = A.R[3 * p]; s_sph[wv][i][1] = A.R[3 * p + 1]; s_sph[wv][i][2] = A.R[3 * p + 2];
      s_sph[wv][i][3] = A.amap[p];
    }
  }
  __syncthreads();
  bool listed = false;
  if (staged && brick == b0) {
#pragma unroll 4
    for (int i = 0; i < c0; ++i) test(s_id[wv][i], s_sph[wv][i][0], s_sph[wv][i][1], s_sph[wv][i][2], s_sph[wv][i][3]);
    listed = true;
  } else if (use_lists) {
    const int cnt = A.bt_cnt[brick];
    if (cnt <= TSLOT) {
      const int32_t *key = A.bt_key + (size_t)brick * TSLOT;
      for (int i = 0; i < cnt; ++i) test_mem(key[i]);
      listed = true;
    }
  }
  if (A.n > 0 && !listed) {
    const Cells &C = A.C;
    int ccy = (int)floor(py * C.iy);
    ccy = ccy < 0 ? 0 : (ccy >= C.ny ? C.ny - 1 : ccy);
    int ccz = (int)floor((double)z * C.iz);
    ccz = ccz < 0 ? 0 : (ccz >= C.nz ? C.nz - 1 : ccz);
    const int zn = C.nz >= 3 ? 3 : C.nz, xn = C.nx >= 3 ? 3 : C.nx;
    for (int dy = -1; dy <= 1; ++dy) {
      int ny = ccy + dy;
      double xs = px;
      if (ny < 0) { ny += C.ny; xs = px + bx.s; }
      else if (ny >= C.ny) { ny -= C.ny; xs = px - bx.s; }
      xs = xs - bx.Lx * floor(xs / bx.Lx);
      int ccx = (int)floor(xs * C.ix);
      ccx = ccx < 0 ? 0 : (ccx >= C.nx ? C.nx - 1 : ccx);
      for (int iz = 0; iz < zn; ++iz) {
        int nz = C.nz >= 3 ? ccz + iz - 1 : iz;
        nz = nz < 0 ? nz + C.nz : (nz >= C.nz ? nz - C.nz : nz);
        for (int ix = 0; ix < xn; ++ix) {
          int nx = C.nx >= 3 ? ccx + ix - 1 : ix;
          nx = nx < 0 ? nx + C.nx : (nx >= C.nx ? nx - C.nx : nx);
          const int c = nx + C.nx * (ny + C.ny * nz);
          for (int t = A.cell_start[c]; t < A.cell_start[c + 1]; ++t) test_mem(A.cell_ids[t]);
        }
      }
    }
  }
  if (!live) return;
  if (clash) atomicOr(A.flags, 1);
  A.gown[idx] = owner;
  if (!A.values || owner >= 0) return;
  if (g == 0) ghost_values<0, ST, CT>(A, bx, x, z);
  else ghost_values<1, ST, CT>(A, bx, x, z);
}

hipError_t launch_ghosts(Sim *s, const Box &b, int32_t *gown_out, void *gval_out, int values, const Clock *clk,
                         int lists) {
  GhostArgs A;
  A.bt_key = s->bt_key; A.bt_cnt = s->bt_cnt;
  A.lists = lists && s->n > 0;
  A.bxn = s->bxn; A.byn = s->byn; A.BZ = s->BZ;
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
__global__ void k_clock(const ClockEntry *tab, Clock *clk, int reset) {
  if (threadIdx.x != 0) return;
  if (reset) {
    clk->idx = 0;
    return;
  }
  const int i = clk->idx;
  clk->cur = tab[i < CLK_CAP ? i : CLK_CAP - 1];
  clk->idx = i + 1;
}

hipError_t launch_clock(Sim *s, int reset) {
  hipLaunchKernelGGL(k_clock, dim3(1), dim3(64), 0, s->stream, s->clk_tab, s->clk, reset);
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
