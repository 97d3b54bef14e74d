// susp_impl.h -- internal declarations of the MI355X suspension library (not installed).
//
// Device layout of one simulation (all carved from one 256-byte aligned block):
//   populations   2 x 19 planes x nodes, storage type (double | float | half), each plane
//                 padded to 256 B; a plane holds deviations d_q = n_q - w_q rho0 (FP16:
//                 d_q / w_q * 2^k) of the post-collision state, x fastest.
//   owner map     nodes int32 (sphere id, -1 fluid), updated in place
//   ghost planes  owner int32 [2][lz][lx]; values [2][5][lz][lx] in compute precision
//   particles     FP64 arrays (positions, velocities, spins, quaternions, radii, ...)
//   lists         cell list, fixed-capacity neighbour lists (NCAP per sphere), spring
//                 history per neighbour entry
//   reductions    per-block fluid stress partials, per-sphere hydrodynamic and pair-stress
//                 accumulators, global stress/G' accumulators, flags
#pragma once
#include <hip/hip_runtime.h>
#include "../../include/susp.h"
#include <hip/hip_fp16.h>
#include <stdint.h>
#include <stddef.h>
#include <string.h>

namespace susp {

constexpr int NQ = 19;
constexpr int NCAP = 48;        // neighbour capacity per sphere
constexpr int HYD = 13;         // F[3] T[3] S[6] nlinks  (per-sphere hydrodynamic sums)
// scales of the two words of the per-sphere fixed-point link sums: hi 2^-FXH, lo 2^-FXL
constexpr int FXH = 20, FXL = 68;
constexpr int PST = 18;         // lubrication, contact, DLVO stress partials (6 each)
// acc (FP64): [0,30) stress of the last step, [30,60) stress sums, 60 their count, 61 sum
// sigma_xy cos, 62 sum sigma_xy sin, 63 observation steps, 64 mass ledger, 65 fluid mass of
// the last step, 66 reference of the conserved fluid mass + ledger, 67 reference taken (1),
// 68 the ledger that pairs with the fluid mass of the last step;
// from ACC_PART on, the partial sums of the stress reduction (RED_BLOCKS x RED_W)
constexpr int RED_BLOCKS = 128;
constexpr int RED_W = 40;
constexpr int ACC_PART = 128;
constexpr int ACC_DOUBLES = ACC_PART + RED_BLOCKS * RED_W;
// largest drift of the fluid mass + ledger, relative to the box's mass, before FL_MASS.  The
// sum is exact for separated spheres (each lattice line's entry and exit links pair up), but
// where two mapped spheres touch node to node the lines running from one into the other lose
// their pairs, and the moving boundaries leak mass slowly: ~1.5-3e-4 of the box per 1000
// steps in dense monolayers and bulk suspensions, in the oracle alike.  The check is for
// runs going wrong, whose drift grows much faster.
constexpr double MASS_TOL = 1e-2;
// instability flags (SUSP_EUNSTABLE)
constexpr int FL_OVERLAP = 1, FL_NONFINITE = 2, FL_NEIGHBOURS = 4, FL_LINKS = 8, FL_JUMP = 16,
              FL_FLUID = 32, FL_MASS = 64;
// the flags block (64 int32) also holds, from word FL_HEALTH on, the health counters: fluid
// node-steps above 0.3 c_s (uint64) and the largest u^2 seen (float bits)
constexpr int FL_HEALTH = 32;
// word of the flags block that counts the finished blocks of the stress reduction
constexpr int FL_REDCNT = 48;
// Link values: each population buffer ends in LINK_CAP elements per node of every 64 x 4 x 4
// brick (of its storage type) that hold the step's bounce-back values, row by row; the record
// of a node (lrec) holds its link directions (bits 1-18), solid (bit 19) and the offset of its
// first value in its row's run (bits 20-31); lrow holds the first value of each 64-node row.
constexpr int LINK_CAP = 5;
// link values a population buffer holds: LINK_CAP per node of every 64 x 4 x 4 brick
inline size_t link_values(int lx, int ly, int lz) {
  return (size_t)((lx + 63) / 64) * ((ly + 3) / 4) * ((lz + 3) / 4) * 1024 * LINK_CAP;
}
constexpr uint32_t REC_SOLID = 1u << 19;
constexpr int REC_OFF = 20;

// D3Q19: 0 rest, 1..6 axes, 7..18 face diagonals; opposite of odd q is q+1.
__host__ __device__ constexpr int cx(int q) {
  return q == 1 || q == 7 || q == 9 || q == 11 || q == 13 ? 1
       : q == 2 || q == 8 || q == 10 || q == 12 || q == 14 ? -1 : 0;
}
__host__ __device__ constexpr int cy(int q) {
  return q == 3 || q == 7 || q == 10 || q == 15 || q == 17 ? 1
       : q == 4 || q == 8 || q == 9 || q == 16 || q == 18 ? -1 : 0;
}
__host__ __device__ constexpr int cz(int q) {
  return q == 5 || q == 11 || q == 14 || q == 15 || q == 18 ? 1
       : q == 6 || q == 12 || q == 13 || q == 16 || q == 17 ? -1 : 0;
}
__host__ __device__ constexpr int opp(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }
__host__ __device__ constexpr double wq(int q) { return q == 0 ? 1.0 / 3.0 : (q <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }
// slot of q among the five directions crossing the y boundary (c_y = +1 or -1)
__host__ __device__ constexpr int gslot(int q) {
  return q == 3 || q == 4 ? 0 : q == 7 || q == 8 ? 1 : q == 10 || q == 9 ? 2 : q == 15 || q == 16 ? 3 : 4;
}
__host__ __device__ constexpr int gdir(int g, int m) {  // g=0: c_y=+1 set, g=1: c_y=-1 set
  return g == 0 ? (m == 0 ? 3 : m == 1 ? 7 : m == 2 ? 10 : m == 3 ? 15 : 17)
                : (m == 0 ? 4 : m == 1 ? 8 : m == 2 ? 9 : m == 3 ? 16 : 18);
}

// Box and Lees-Edwards state for geometric predicates (FP64, fixed operation order).
struct Box {
  int lx, ly, lz;
  double Lx, Ly, Lz;
  double s;    // offset of the image above (x shift of the box at +Ly)
  double ule;  // its velocity
};

// Minimum-image displacement d = point - particle; k = image index of the particle
// (its image sits at R + k (s, Ly, 0) and moves with U + k ule x).
__host__ __device__ inline void minimage(const Box &b, double dx, double dy, double dz,
                                         double &ox, double &oy, double &oz, int &k) {
  k = 0;
  if (dy > 0.5 * b.Ly) { dy -= b.Ly; dx -= b.s; k = 1; }
  else if (dy < -0.5 * b.Ly) { dy += b.Ly; dx += b.s; k = -1; }
  // at most a few periods apart for finite input; the bound keeps non-finite input finite-time
  for (int it = 0; it < 4 && dx > 0.5 * b.Lx; ++it) dx -= b.Lx;
  for (int it = 0; it < 4 && dx < -0.5 * b.Lx; ++it) dx += b.Lx;
  for (int it = 0; it < 4 && dz > 0.5 * b.Lz; ++it) dz -= b.Lz;
  for (int it = 0; it < 4 && dz < -0.5 * b.Lz; ++it) dz += b.Lz;
  ox = dx; oy = dy; oz = dz;
}

// Storage of population deviations.  FP16 keeps h = half(d / w_q * 2^k); the factors
// 2^k / w_q (= 2^k times 3, 18 or 36) and w_q 2^-k are formed exactly from the scalars
// up = 2^k and dn = 2^-k.
struct H16 {
  float up, dn;
};
template <class ST> struct Store;
template <> struct Store<double> {
  using CT = double;
  __device__ static double ld(const double *p, size_t i, int, H16) { return p[i]; }
  __device__ static void st(double *p, size_t i, double v, int, H16) { p[i] = v; }
};
template <> struct Store<float> {
  using CT = float;
  __device__ static float ld(const float *p, size_t i, int, H16) { return p[i]; }
  __device__ static void st(float *p, size_t i, float v, int, H16) { p[i] = v; }
};
template <> struct Store<__half> {
  using CT = float;
  __device__ static float ld(const __half *p, size_t i, int q, H16 h) {
    return __half2float(p[i]) * ((float)wq(q) * h.dn);
  }
  __device__ static void st(__half *p, size_t i, float v, int q, H16 h) {
    p[i] = __float2half_rn(v * ((float)(1.0 / wq(q)) * h.up));
  }
};

// Shear-protocol values of one lattice step t (eq. 16 or simple shear): LE offset and
// velocity at t and t+1, and the G', G'' quadrature weights of the step.  The host writes a
// table of them ahead of a run of steps; k_clock copies entry idx to cur at the start of
// each step, so that a recorded sequence of steps (a HIP graph) replays with fixed
// kernel arguments.
struct ClockEntry {
  double s, ule, s1, ule1, gcos, gsin;
  double uw, uw1;  // walls: speed of the top wall at t and t+1 (the bottom one moves at -uw)
  int32_t gphase, pad;
};
struct Clock {
  ClockEntry cur;
  int32_t idx, pad;
};
constexpr int CLK_CAP = 4096;  // steps per table upload
constexpr int PROF_EV = 3;     // timing events per profiled step

// Box of the current step (next = 0: offset s, velocity ule) or of the next one (s1, ule1)
// from the device clock; without a clock the box is used as given.
__device__ inline Box clock_box(Box b, const Clock *c, int next) {
  if (c) {
    b.s = next ? c->cur.s1 : c->cur.s;
    b.ule = next ? c->cur.ule1 : c->cur.ule;
  }
  return b;
}

// Cell grid for the neighbour search.
struct Cells {
  int nx, ny, nz;
  double ix, iy, iz;  // cells per unit length (n / L)
};

struct Sim;

// ---- multi-job launches ----
// A step's kernels can run for many simulations at once: one launch whose work-groups
// [pre[j], pre[j+1]) belong to job j, with job j's arguments in tab[j].  Each kernel body
// takes its work-group index within its job; the one-job kernel passes blockIdx.x.
// Work-group of a multi-job launch -> its job (pre ascends, pre[0] = 0, nj jobs).
__device__ inline int multi_job(const int32_t *__restrict__ pre, int nj, int b) {
  int lo = 0, hi = nj - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}
// The multi-job kernel of a body: the job's arguments are read from its table entry.
#define SUSP_MULTI_BODY(ARGS, BODY)                            \
  const int mj_ = multi_job(pre, nj, (int)blockIdx.x);         \
  BODY(tab[mj_], (int)blockIdx.x - pre[mj_])

// Launches of one simulation recorded instead of issued (the batch builds its multi-job
// launches from them): the multi-job kernel, the job's work-group count and block size,
// and the argument bytes.
struct Collect {
  struct Rec {
    const void *fn;
    unsigned grid, blk;
    size_t off, sz;
  };
  Rec rec[256];
  int nrec;
  char bytes[256 * 512];
  size_t used;
  int overflow;
  void clear() { nrec = 0; used = 0; overflow = 0; }
  hipError_t add(const void *fn, unsigned grid, unsigned blk, const void *a, size_t sz) {
    const size_t al = (sz + 15) / 16 * 16;
    if (nrec == 256 || used + al > sizeof bytes) { overflow = 1; return hipErrorInvalidValue; }
    memcpy(bytes + used, a, sz);
    rec[nrec++] = Rec{fn, grid, blk, used, sz};
    used += al;
    return hipSuccess;
  }
};

// ---- launchers (fluid.hip) ----
hipError_t launch_init_populations(Sim *s);
// cleared: the planes were cleared by the step's clock kernel
hipError_t launch_ghosts(Sim *s, const Box &b, int32_t *gown_out, int32_t *gcnt, void *gval_out, int values,
                         const Clock *clk, int cleared);
hipError_t launch_links(Sim *s, const Box &b);
hipError_t launch_lbm(Sim *s, const Box &b);
hipError_t launch_pop_convert(Sim *s, double *dev64, int to_storage);
hipError_t launch_pop_plane(Sim *s, double *dev64, int q, int to_storage);
hipError_t launch_link_enum(Sim *s, const int32_t *gown, int32_t *out /*[nodes]*/, int q);
// ---- launchers (particles.hip) ----
hipError_t launch_cells(Sim *s, int32_t *cell_start, int32_t *cell_ids, int32_t *scratch);
hipError_t launch_pairs(Sim *s, const Box &b);
hipError_t launch_pair_rev(Sim *s);
hipError_t launch_substep(Sim *s, const Box &b, int sub);
hipError_t launch_map_full(Sim *s, const Box &b);
hipError_t launch_map_update(Sim *s, const Box &b, int phase);
hipError_t launch_stress(Sim *s);
hipError_t launch_contact_sample(Sim *s);
hipError_t launch_walls(Sim *s);
hipError_t launch_wall_force(Sim *s);
hipError_t launch_contact_final(Sim *s, double *out);
hipError_t launch_fill_i32(int32_t *p, size_t n, int32_t v, hipStream_t st);
hipError_t launch_clock(Sim *s, int reset);
hipError_t launch_fill_f64(double *p, size_t n, double v, hipStream_t st);

struct Sim {
  // problem
  int lx, ly, lz, precision;
  int64_t nodes;
  size_t plane;  // elements per population plane (padded)
  int n;
  double tau, rho0;
  double map_ratio, rho_p;
  double m0, kn, kt, eta_n, lub_delta, F0, lambda, eta0, a_min, a_max;
  double mu, lub_hc, pair_cutoff;
  int lub_sub, n_sub, quasi2d;
  int shear_kind;
  double gamma_dot, g0_I, g0_F, theta;
  int period, ncyc_I, ncyc_F;
  int fp16_exp;
  int collision;           // 0 BGK, 1 multi-eigenvalue (tau shear, tau_bulk, tau_ghost)
  int lub_implicit;        // Jacobi sweeps of the implicit squeeze terms per substep (0: off)
  double *lb, *uimp;       // [n][3] their right-hand sides and scratch velocities
  int boundary;            // 0 Lees-Edwards, 1 moving walls with wall spheres
  int32_t *wmem;           // [n] 0 free, 1 bottom wall, 2 top wall
  double *wfs;             // [n][3] force on each wall sphere this step (hydro + pair mean)
  double *wpart;           // [ghost blocks][6] flat-wall momentum per block
  double *wacc;            // [8] summed force on the bottom, top wall; steps
  double tau_bulk, tau_ghost;
  H16 h16;                 // FP16 storage scale 2^k and its inverse
  Cells cells;
  int ncell;
  int bxn, byn, bzn, BY, BZ, nbricks;  // lattice-kernel bricks of 64 x BY x BZ nodes
  // device block
  void *block;
  int owns_block;
  hipStream_t stream;
  int device;  // the device current when the simulation was created (its block and stream)
  // populations
  void *f[2];
  int cur;  // index of the buffer holding the current state
  int32_t *own;  // owner map: sphere id of every node, -1 fluid
  uint32_t *lrec;  // [nodes] link record of every node (k_links), read by k_stream
  int32_t *lrow;   // [lx/64 rounded up * ly * lz] first link value of each 64-node row
  int32_t *gown;
  int32_t *gcnt;  // [2][lz][lx] spheres covering each ghost point
  void *gval;
  // particles (FP64)
  double *R[2], *U[2], *W[2], *Q[2];
  int pcur;  // current particle buffer
  double *R0;
  double *a, *m, *I, *amap;
  double *hyd[2];
  int hcur;
  unsigned long long *hacc;  // [n][HYD][2] fixed-point link sums of the step (link phase)
  double *pst;   // [n][PST]
  double *dp;    // [n][8] cover/uncover momentum, angular momentum, mass
  // lists
  int32_t *cell_start, *cell_ids, *cell_scr;
  int32_t *ncnt[2], *nj[2];  // neighbour count [n], neighbour ids [n][NCAP]
  int lcur;                  // list of the last step
  double *hxi[3];            // spring vector per entry [n][NCAP][3]
  int32_t *hon[3];           // contact flag per entry
  int32_t *hstart;           // contact at the start of the step per entry
  int32_t *rev;              // per entry: entry (of the lower id) holding the pair's history
  int hfin;                  // history buffer holding the final state of the last step
  // contact statistics (cbins > 0): records of the last substep's contacts, per-step
  // partial sums and the running sums since the last read-out
  int cbins;
  int cchunks;               // sphere chunks of 256 per bin in the partial sums
  double cgeo[2];            // mean radius, volume (monolayer: area) fraction
  double *crec;              // [n][NCAP][4] n_x, n_y, F_nor, F_tan of the entry's contact
  int32_t *cflag;            // [n][NCAP] 1 if the entry holds a contact record, else 0
  double *cpart;             // [(cbins + 1) * cchunks][6]
  double *cacc;              // [cbins + 1][6] sums, then the total stress sum [6], samples
  double *cout;              // [5 * cbins + 12] read-out staging
  // reductions
  double *pin;    // [nbricks][8] fluid stress partials (6), mass deviation, fluid nodes
  double *acc;    // sig_last[30] sig_sum[30] count gp_cos gp_sin gp_count ledger, fluid mass
                  // deviation, conserved-mass reference and its flag; then reduction partials
  int32_t *flags;
  // clock
  int64_t step;
  ClockEntry *clk_tab;   // device table of the next steps' protocol values
  Clock *clk;            // device: current entry and table cursor
  ClockEntry *clk_host;  // host staging of the table
  // recorded steps replayed as one HIP graph (streams other than the null stream)
  int graph_on;            // pairs of steps per graph (0: no graphs)
  hipGraphExec_t gexec;    // null until recorded
  int gparity;             // cur ^ 2 lcur ^ 4 hcur ^ 8 pcur ^ 16 hfin at recording
  // optional timing of the lattice kernel with HIP events on the simulation's stream
  int prof_on;
  int prof_used, prof_cap;
  hipEvent_t *prof_ev;  // [PROF_EV * prof_cap]: before k_links, before k_stream, after it
  // non-null: launches of the step are recorded here (multi-job batches), not issued
  Collect *col;
};

// Issue a kernel of one simulation, or record it for a multi-job launch.
template <class A>
inline hipError_t dispatch(Sim *s, void (*one)(A), void (*multi)(const A *, const int32_t *, int), unsigned grid,
                           unsigned blk, const A &args) {
  if (s->col) return s->col->add((const void *)multi, grid, blk, &args, sizeof(A));
  void *kp[] = {(void *)&args};
  return hipLaunchKernel((const void *)one, dim3(grid), dim3(blk), kp, 0, s->stream);
}
// Launchers of kernels that have no multi-job form refuse to record.
#define SUSP_NO_COLLECT(s) \
  do { if ((s)->col) return hipErrorNotSupported; } while (0)

// ---- stepping helpers shared by the single-simulation and batch entry points (api.hip) ----
int launch_steps(susp_sim *h, int64_t nsteps);
Sim &sim_of(susp_sim *h);
bool multi_ok(const susp_sim *h);
int record_two_steps(susp_sim *h, Collect *c);
int prepare_run(susp_sim *h, int m);
void advance_steps(susp_sim *h, int m);
int step_parity(const susp_sim *h);
int check_flags(susp_sim *h);
int set_error(int code, const char *msg);

}  // namespace susp
