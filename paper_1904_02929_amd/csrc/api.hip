// api.hip -- host side of the C ABI declared in include/susp.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/susp.h"
#include "susp_impl.h"

using namespace susp;

struct susp_sim {
  Sim s;
};

static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(SUSP_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

extern "C" const char *susp_last_error(void) { return g_err.c_str(); }

extern "C" void susp_default_params(susp_params *p) {
  memset(p, 0, sizeof *p);
  p->precision = SUSP_FP32;
  p->tau = 1.0;
  p->rho0 = 1.0;
  p->map_ratio = 0.95;
  p->rho_p = 1.0;
  p->tau_bulk = 1.0;
  p->tau_ghost = 1.0;
  p->kn = -1.0;
  p->kt_ratio = 0.5;
  p->mu = 1.0;
  p->eta_n = -1.0;
  p->lub_delta = -1.0;
  p->lub_hc = 0.5;
  p->lub_subtract_hc = 1;
  p->F0 = -1.0;
  p->debye_lambda = -1.0;
  p->pair_cutoff = 1.0;
  p->n_sub = 8;
  p->period = 1;
  p->fp16_exp = 10;
}

// ---------------------------------------------------------------------------------------
// Shear protocol: offset and sliding velocity of the image box above at step t
// (simple shear, or eq. (16) with the amplitude switched after ncyc_I periods).
static void le_protocol(const Sim &s, int64_t t, double *off, double *ule) {
  const double Lx = s.lx, Ly = s.ly;
  if (s.shear_kind == 1) {
    const double u = s.gamma_dot * Ly;
    const double x = (double)t * u;
    *off = x - Lx * floor(x / Lx);
    *ule = u;
  } else if (s.shear_kind == 2) {
    const int64_t P = s.period;
    const int64_t tI = (int64_t)s.ncyc_I * P;
    const double g0 = t < tI ? s.g0_I : s.g0_F;
    const int64_t tp = t < tI ? t : t - tI;
    const double om = 2.0 * 3.14159265358979323846 / (double)P;
    const double ph = om * (double)tp + s.theta;
    const double gam = g0 * (cos(s.theta) - cos(ph));
    const double gdot = om * g0 * sin(ph);
    const double x = Ly * gam;
    *off = x - Lx * floor(x / Lx);
    *ule = Ly * gdot;
  } else {
    *off = 0.0;
    *ule = 0.0;
  }
}

// Lees-Edwards offset and sliding velocity of step t (none with walls)
static void protocol(const Sim &s, int64_t t, double *off, double *ule) {
  if (s.boundary == 1) { *off = 0.0; *ule = 0.0; return; }
  le_protocol(s, t, off, ule);
}

// Walls: speed of the top wall, half the velocity difference L_y gamma_dot(t) across the box
static double wall_speed(const Sim &s, int64_t t) {
  double off, ule;
  le_protocol(s, t, &off, &ule);
  return 0.5 * ule;
}

static Box make_box(const Sim &s, double off, double ule) {
  Box b;
  b.lx = s.lx; b.ly = s.ly; b.lz = s.lz;
  b.Lx = s.lx; b.Ly = s.ly; b.Lz = s.lz;
  b.s = off; b.ule = ule;
  return b;
}

// ---------------------------------------------------------------------------------------
static int resolve(const susp_params *p, Sim &s) {
  if (!p) return fail(SUSP_EINVAL, "params is NULL");
  if (p->lx < 8 || p->ly < 8 || p->lz < 8) return fail(SUSP_EINVAL, "lattice must be at least 8^3");
  if ((int64_t)p->lx * p->ly * p->lz > (int64_t)1 << 31)
    return fail(SUSP_EINVAL, "lattice larger than 2^31 nodes");
  if (p->precision < 0 || p->precision > 2) return fail(SUSP_EINVAL, "bad precision");
  if (!(p->tau > 0.5)) return fail(SUSP_EINVAL, "tau must exceed 1/2");
  if (!(p->rho0 > 0)) return fail(SUSP_EINVAL, "rho0 must be positive");
  if (p->n < 0) return fail(SUSP_EINVAL, "negative sphere count");
  if (p->n > 0 && (!p->pos || !p->radius)) return fail(SUSP_EINVAL, "pos/radius missing");
  if (p->n_sub < 1) return fail(SUSP_EINVAL, "n_sub must be >= 1");
  if (p->shear_kind < 0 || p->shear_kind > 2) return fail(SUSP_EINVAL, "bad shear_kind");
  if (p->shear_kind == 2 && p->period < 1) return fail(SUSP_EINVAL, "period must be >= 1");
  if (!(p->map_ratio > 0 && p->map_ratio <= 1)) return fail(SUSP_EINVAL, "map_ratio in (0,1]");
  if (!(p->pair_cutoff >= p->lub_hc) || !(p->pair_cutoff > 0))
    return fail(SUSP_EINVAL, "pair_cutoff must be positive and >= lub_hc");
  s.lx = p->lx; s.ly = p->ly; s.lz = p->lz;
  s.precision = p->precision;
  s.nodes = (int64_t)p->lx * p->ly * p->lz;
  s.plane = (size_t)((s.nodes + 255) / 256 * 256);
  {
    // the lattice kernel addresses one population array with 32-bit byte offsets
    const size_t es = p->precision == 0 ? 8 : p->precision == 1 ? 4 : 2;
    if (((size_t)NQ * s.plane + link_values(p->lx, p->ly, p->lz)) * es > 0xffffffffull)
      return fail(SUSP_EINVAL, "one population array would exceed 4 GiB (%zu nodes, %zu-byte storage)",
                  (size_t)s.nodes, es);
  }
  s.n = p->n;
  s.tau = p->tau; s.rho0 = p->rho0;
  s.map_ratio = p->map_ratio; s.rho_p = p->rho_p;
  const double PI = 3.14159265358979323846;
  double amin = 0, amax = 0, msum = 0;
  for (int i = 0; i < p->n; ++i) {
    const double a = p->radius[i];
    if (!(a > 0)) return fail(SUSP_EINVAL, "radius %d not positive", i);
    if (i == 0 || a < amin) amin = a;
    if (i == 0 || a > amax) amax = a;
    msum += p->rho_p * (4.0 / 3.0) * PI * a * a * a;
    for (int c = 0; c < 3; ++c) {
      const double L = c == 0 ? p->lx : (c == 1 ? p->ly : p->lz);
      const double x = p->pos[3 * i + c];
      if (!(x >= 0.0 && x < L)) return fail(SUSP_EINVAL, "sphere %d outside the box", i);
    }
  }
  s.a_min = amin; s.a_max = amax;
  s.m0 = p->n > 0 ? msum / p->n : 0.0;
  s.kn = p->kn > 0 ? p->kn : 0.36 * s.m0;  // dt = 0.6 sqrt(m0/kn), dt = 1
  s.kt = p->kt_ratio * s.kn;
  s.eta_n = p->eta_n >= 0 ? p->eta_n : sqrt(s.m0 * s.kn);
  s.lub_delta = p->lub_delta >= 0 ? p->lub_delta : 0.01 * amin;
  s.lambda = p->debye_lambda > 0 ? p->debye_lambda : 0.02 * amin;
  s.F0 = p->F0 >= 0 ? p->F0 : 2e-4 * s.kn;
  s.eta0 = p->rho0 * (p->tau - 0.5) / 3.0;
  s.mu = p->mu; s.lub_hc = p->lub_hc; s.pair_cutoff = p->pair_cutoff;
  s.lub_sub = p->lub_subtract_hc; s.n_sub = p->n_sub; s.quasi2d = p->quasi2d;
  s.shear_kind = p->shear_kind;
  s.gamma_dot = p->gamma_dot; s.g0_I = p->g0_I; s.g0_F = p->g0_F; s.theta = p->theta;
  s.period = p->period; s.ncyc_I = p->ncyc_I; s.ncyc_F = p->ncyc_F;
  s.fp16_exp = p->fp16_exp;
  if (p->contact_bins < 0 || p->contact_bins > 360) return fail(SUSP_EINVAL, "contact_bins must be in [0, 360]");
  if (p->collision < 0 || p->collision > 1) return fail(SUSP_EINVAL, "collision must be 0 or 1");
  if (p->collision == 1 && !(p->tau_bulk > 0.5 && p->tau_ghost > 0.5))
    return fail(SUSP_EINVAL, "tau_bulk and tau_ghost must exceed 1/2");
  if (p->lub_implicit < 0 || p->lub_implicit > 64) return fail(SUSP_EINVAL, "lub_implicit must be in [0, 64]");
  s.lub_implicit = p->lub_implicit;
  if (p->boundary < 0 || p->boundary > 1) return fail(SUSP_EINVAL, "boundary must be 0 or 1");
  s.boundary = p->boundary;
  if (p->boundary == 1 && p->wall) {
    // a wall sphere keeps pair_cutoff / 2 from its own face, so that the two walls never
    // meet through the periodic image in y
    for (int i = 0; i < p->n; ++i) {
      const int m = p->wall[i];
      const double y = p->pos[3 * i + 1], a = p->radius[i], h = 0.5 * p->pair_cutoff;
      if (m < 0 || m > 2) return fail(SUSP_EINVAL, "wall membership %d of sphere %d not in 0..2", m, i);
      if ((m == 1 && !(y > a + h)) || (m == 2 && !(y < p->ly - a - h)))
        return fail(SUSP_EINVAL, "wall sphere %d closer than pair_cutoff / 2 to its face", i);
    }
  }
  s.collision = p->collision;
  s.tau_bulk = p->collision ? p->tau_bulk : p->tau;
  s.tau_ghost = p->collision ? p->tau_ghost : p->tau;
  s.cbins = p->contact_bins;
  s.cchunks = p->n > 0 ? (p->n + 255) / 256 : 1;
  {
    // eqs. 26-27: mean radius and the volume (monolayer: area) fraction of the spheres
    double as = 0.0, a2 = 0.0, a3 = 0.0;
    for (int i = 0; i < p->n; ++i) {
      const double a = p->radius[i];
      as += a;
      a2 += PI * a * a;
      a3 += (4.0 / 3.0) * PI * a * a * a;
    }
    s.cgeo[0] = p->n > 0 ? as / p->n : 0.0;
    s.cgeo[1] = p->quasi2d ? a2 / ((double)p->lx * p->ly) : a3 / ((double)p->lx * p->ly * p->lz);
  }
  if (p->precision == 2 && (p->fp16_exp < -20 || p->fp16_exp > 20))
    return fail(SUSP_EINVAL, "fp16_exp out of [-20, 20]");
  s.h16.up = (float)ldexp(1.0, p->fp16_exp);  // deviation -> storage: d / w_q * 2^k
  s.h16.dn = (float)ldexp(1.0, -p->fp16_exp);
  // cell grid: width >= 2 a_max + cutoff, at least 3 cells across the sliding direction
  const double rc = 2.0 * amax * (p->n > 0 ? 1.0 : 0.0) + p->pair_cutoff + 1e-6;
  const int L[3] = {p->lx, p->ly, p->lz};
  int nc[3];
  for (int c = 0; c < 3; ++c) {
    nc[c] = (int)floor(L[c] / rc);
    if (nc[c] < 1) nc[c] = 1;
    if (nc[c] > 64) nc[c] = 64;
  }
  if (p->n > 0 && nc[1] < 3)
    return fail(SUSP_EINVAL, "ly must hold 3 cells of 2 a_max + pair_cutoff");
  const double amap = p->map_ratio * amax;
  if (p->n > 0 && (p->lx <= 2 * amap || p->lz <= 2 * amap))
    return fail(SUSP_EINVAL, "lx and lz must exceed the mapped diameter");
  s.cells.nx = nc[0]; s.cells.ny = nc[1]; s.cells.nz = nc[2];
  s.cells.ix = nc[0] / (double)p->lx;
  s.cells.iy = nc[1] / (double)p->ly;
  s.cells.iz = nc[2] / (double)p->lz;
  s.ncell = nc[0] * nc[1] * nc[2];
  // bricks of 64 x BY x BZ nodes for the stream kernel.  With spheres the default is 64 x 4 x 4,
  // the link kernel's brick, so that one work-group takes both (k_lattice); without them at most
  // 64 x 8 x 8, smaller until at least 2048 of them spread over the 256 compute units
  s.bxn = (p->lx + 63) / 64;
  auto nbr = [&]() { return s.bxn * ((p->ly + s.BY - 1) / s.BY) * ((p->lz + s.BZ - 1) / s.BZ); };
  if (p->brick_y || p->brick_z) {
    if (p->brick_y < 4 || p->brick_y % 4 || p->brick_y > 1024 || p->brick_z < 1 || p->brick_z > 1024)
      return fail(SUSP_EINVAL, "brick_y must be a positive multiple of 4 and brick_z positive (<= 1024)");
    s.BY = p->brick_y; s.BZ = p->brick_z;
  } else if (p->n > 0) {
    s.BY = 4; s.BZ = 4;
  } else {
    s.BY = 8; s.BZ = 8;
    while (nbr() < 2048 && (s.BY > 4 || s.BZ > 1)) {
      if (s.BZ >= s.BY && s.BZ > 1) s.BZ /= 2;
      else if (s.BY > 4) s.BY /= 2;
      else s.BZ /= 2;
    }
  }
  s.byn = (p->ly + s.BY - 1) / s.BY;
  s.bzn = (p->lz + s.BZ - 1) / s.BZ;
  s.nbricks = nbr();
  return SUSP_OK;
}

// Carve (or size) the device block.  With base == NULL only the size is computed.
static size_t carve(Sim &s, char *base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> void * {
    void *p = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    if (bytes == 0) off += 256;
    return p;
  };
  const size_t es = s.precision == 0 ? 8 : (s.precision == 1 ? 4 : 2);
  const size_t cs = s.precision == 0 ? 8 : 4;
  const size_t n = (size_t)s.n;
  // each population buffer ends in the link values of the steps that read it
  for (int b = 0; b < 2; ++b) s.f[b] = take((NQ * s.plane + link_values(s.lx, s.ly, s.lz)) * es);
  // the ghost owner planes right after the owner map: the lattice kernel reads both through
  // one buffer resource
  s.own = (int32_t *)take((size_t)s.nodes * 4);
  s.gown = (int32_t *)take((size_t)2 * s.lx * s.lz * 4);
  s.gval = take((size_t)2 * 5 * s.lx * s.lz * cs);
  s.gcnt = (int32_t *)take((size_t)2 * s.lx * s.lz * 4);
  s.lrec = (uint32_t *)take((size_t)s.nodes * 4);
  s.lrow = (int32_t *)take((size_t)((s.lx + 63) / 64) * s.ly * s.lz * 4);
  for (int b = 0; b < 2; ++b) {
    s.R[b] = (double *)take(n * 3 * 8);
    s.U[b] = (double *)take(n * 3 * 8);
    s.W[b] = (double *)take(n * 3 * 8);
    s.Q[b] = (double *)take(n * 4 * 8);
    s.hyd[b] = (double *)take(n * HYD * 8);
  }
  s.R0 = (double *)take(n * 3 * 8);
  s.hacc = (unsigned long long *)take(n * HYD * 2 * 8);
  s.a = (double *)take(n * 8);
  s.m = (double *)take(n * 8);
  s.I = (double *)take(n * 8);
  s.amap = (double *)take(n * 8);
  s.pst = (double *)take(n * PST * 8);
  s.dp = (double *)take(n * 8 * 8);
  s.cell_start = (int32_t *)take((size_t)(s.ncell + 1) * 4);
  s.cell_ids = (int32_t *)take(n * 4);
  s.cell_scr = (int32_t *)take((size_t)s.ncell * 4);
  for (int b = 0; b < 2; ++b) {
    s.ncnt[b] = (int32_t *)take(n * 4);
    s.nj[b] = (int32_t *)take(n * NCAP * 4);
    s.hxi[b] = (double *)take(n * NCAP * 3 * 8);
    s.hon[b] = (int32_t *)take(n * NCAP * 4);
  }
  s.hstart = (int32_t *)take(n * NCAP * 4);
  s.rev = (int32_t *)take(n * NCAP * 4);
  if (s.lub_implicit > 0) {
    s.lb = (double *)take(n * 3 * 8);
    s.uimp = (double *)take(n * 3 * 8);
  }
  if (s.boundary == 1) {
    s.wmem = (int32_t *)take(n * 4);
    s.wfs = (double *)take(n * 3 * 8);
    s.wpart = (double *)take((size_t)((2 * s.lx * s.lz + 255) / 256) * 6 * 8);
    s.wacc = (double *)take(8 * 8);
  }
  if (s.cbins > 0) {
    s.crec = (double *)take(n * NCAP * 4 * 8);
    s.cflag = (int32_t *)take(n * NCAP * 4);
    s.cpart = (double *)take((size_t)(s.cbins + 1) * s.cchunks * 6 * 8);
    s.cacc = (double *)take((size_t)((s.cbins + 1) * 6 + 8) * 8);
    s.cout = (double *)take((size_t)(5 * s.cbins + 12) * 8);
  }
  s.pin = (double *)take((size_t)s.nbricks * 8 * 8);
  s.acc = (double *)take((size_t)ACC_DOUBLES * 8);
  s.flags = (int32_t *)take(256);
  s.clk_tab = (ClockEntry *)take((size_t)CLK_CAP * sizeof(ClockEntry));
  s.clk = (Clock *)take(sizeof(Clock));
  return off;
}

extern "C" size_t susp_footprint_bytes(const susp_params *p) {
  Sim s;
  memset(&s, 0, sizeof s);
  if (resolve(p, s) != SUSP_OK) return 0;
  return carve(s, nullptr);
}

static int reset_mass_reference(Sim &s);

static int remap(Sim &s) {
  // both maps to fluid, then claim the current footprints (no cover/uncover)
  int rc = reset_mass_reference(s);
  if (rc) return rc;
  HIPCHK(launch_fill_i32(s.own, (size_t)s.nodes, -1, s.stream));
  double off, ule;
  protocol(s, s.step, &off, &ule);
  HIPCHK(launch_map_full(&s, make_box(s, off, ule)));
  return SUSP_OK;
}

// The next step takes a new reference for the conserved fluid mass + ledger (the state was
// replaced).
static int reset_mass_reference(Sim &s) {
  HIPCHK(launch_fill_f64(s.acc + 65, 4, 0.0, s.stream));
  return SUSP_OK;
}

static int read_flags(Sim &s, int32_t *out) {
  HIPCHK(hipMemcpyAsync(out, s.flags, 4, hipMemcpyDeviceToHost, s.stream));
  HIPCHK(hipStreamSynchronize(s.stream));
  HIPCHK(launch_fill_i32(s.flags, 1, 0, s.stream));
  return SUSP_OK;
}

extern "C" int susp_create(const susp_params *p, void *stream, void *workspace, size_t ws_bytes,
                           susp_sim **out) {
  if (!out) return fail(SUSP_EINVAL, "out is NULL");
  *out = nullptr;
  susp_sim *h = new susp_sim;
  Sim &s = h->s;
  memset(&s, 0, sizeof s);
  int rc = resolve(p, s);
  if (rc) { delete h; return rc; }
  s.stream = (hipStream_t)stream;
  if (hipGetDevice(&s.device) != hipSuccess) { delete h; return fail(SUSP_EDEVICE, "hipGetDevice"); }
  const size_t need = carve(s, nullptr);
  char *base = nullptr;
  if (workspace) {
    if (ws_bytes < need) { delete h; return fail(SUSP_ENOMEM, "workspace %zu < %zu bytes", ws_bytes, need); }
    if (((uintptr_t)workspace & 255) != 0) { delete h; return fail(SUSP_EINVAL, "workspace not 256-byte aligned"); }
    base = (char *)workspace;
    s.owns_block = 0;
  } else {
    hipError_t e = hipMalloc((void **)&base, need);
    if (e != hipSuccess) { delete h; return fail(SUSP_ENOMEM, "hipMalloc(%zu): %s", need, hipGetErrorString(e)); }
    s.owns_block = 1;
  }
  s.block = base;
  carve(s, base);
  auto bail = [&](int code) { susp_destroy(h); return code; };
  s.clk_host = (ClockEntry *)malloc((size_t)CLK_CAP * sizeof(ClockEntry));
  if (!s.clk_host) return bail(fail(SUSP_ENOMEM, "clock table"));
  if (launch_fill_i32((int32_t *)s.clk, sizeof(Clock) / 4, 0, s.stream)) return bail(fail(SUSP_EDEVICE, "fill"));
  const size_t n = (size_t)s.n;
  if (n) {
    std::vector<double> v(n * 4, 0.0), a(n), m(n), I(n), am(n);
    const double PI = 3.14159265358979323846;
    for (size_t i = 0; i < n; ++i) {
      a[i] = p->radius[i];
      m[i] = p->rho_p * (4.0 / 3.0) * PI * a[i] * a[i] * a[i];
      I[i] = 0.4 * m[i] * a[i] * a[i];
      am[i] = p->map_ratio * a[i];
    }
    // initial velocities; wall spheres move with their wall
    std::vector<double> u0(n * 3, 0.0), w0(n * 3, 0.0);
    std::vector<int32_t> wm(n, 0);
    for (size_t i = 0; i < 3 * n; ++i) {
      if (p->vel) u0[i] = p->vel[i];
      if (p->omega) w0[i] = p->omega[i];
    }
    if (s.boundary == 1 && p->wall) {
      const double uw = wall_speed(s, 0);
      for (size_t i = 0; i < n; ++i) {
        wm[i] = p->wall[i];
        if (wm[i] == 0) continue;
        u0[3 * i] = wm[i] == 2 ? uw : -uw;
        u0[3 * i + 1] = u0[3 * i + 2] = 0.0;
        w0[3 * i] = w0[3 * i + 1] = w0[3 * i + 2] = 0.0;
      }
    }
    if (s.boundary == 1 && (hipMemcpyAsync(s.wmem, wm.data(), n * 4, hipMemcpyHostToDevice, s.stream) ||
                            hipStreamSynchronize(s.stream)))
      return bail(fail(SUSP_EDEVICE, "upload"));
    for (int b = 0; b < 2; ++b) {
      if (hipMemcpyAsync(s.R[b], p->pos, n * 24, hipMemcpyHostToDevice, s.stream)) return bail(fail(SUSP_EDEVICE, "upload"));
      if (hipMemcpyAsync(s.U[b], u0.data(), n * 24, hipMemcpyHostToDevice, s.stream)) return bail(fail(SUSP_EDEVICE, "upload"));
      if (hipMemcpyAsync(s.W[b], w0.data(), n * 24, hipMemcpyHostToDevice, s.stream)) return bail(fail(SUSP_EDEVICE, "upload"));
      for (size_t i = 0; i < n; ++i) v[4 * i] = 1.0;
      if (hipMemcpyAsync(s.Q[b], v.data(), n * 32, hipMemcpyHostToDevice, s.stream)) return bail(fail(SUSP_EDEVICE, "upload"));
      if (hipStreamSynchronize(s.stream)) return bail(fail(SUSP_EDEVICE, "sync"));
    }
    if (hipMemcpyAsync(s.a, a.data(), n * 8, hipMemcpyHostToDevice, s.stream) ||
        hipMemcpyAsync(s.m, m.data(), n * 8, hipMemcpyHostToDevice, s.stream) ||
        hipMemcpyAsync(s.I, I.data(), n * 8, hipMemcpyHostToDevice, s.stream) ||
        hipMemcpyAsync(s.amap, am.data(), n * 8, hipMemcpyHostToDevice, s.stream) ||
        hipStreamSynchronize(s.stream))
      return bail(fail(SUSP_EDEVICE, "upload of radii"));
  }
  s.cur = 0; s.pcur = 0; s.hcur = 0; s.lcur = 0; s.hfin = 0; s.step = 0;
  s.graph_on = 5;
  if (launch_init_populations(&s)) return bail(fail(SUSP_EDEVICE, "init populations"));
  if (launch_fill_i32(s.gown, (size_t)2 * s.lx * s.lz, -1, s.stream)) return bail(fail(SUSP_EDEVICE, "fill"));
  for (int b = 0; b < 2; ++b) {
    if (n && (launch_fill_f64(s.hyd[b], n * HYD, 0.0, s.stream) || launch_fill_i32(s.ncnt[b], n, 0, s.stream) ||
              launch_fill_i32(s.hon[b], n * NCAP, 0, s.stream)))
      return bail(fail(SUSP_EDEVICE, "fill"));
  }
  if (n && launch_fill_i32((int32_t *)s.hacc, n * HYD * 4, 0, s.stream)) return bail(fail(SUSP_EDEVICE, "fill"));
  if (n && (launch_fill_f64(s.pst, n * PST, 0.0, s.stream) || launch_fill_f64(s.dp, n * 8, 0.0, s.stream) ||
            launch_fill_i32(s.hstart, n * NCAP, 0, s.stream)))
    return bail(fail(SUSP_EDEVICE, "fill"));
  if (launch_fill_f64(s.acc, ACC_DOUBLES, 0.0, s.stream) || launch_fill_i32(s.flags, 64, 0, s.stream) ||
      launch_fill_f64(s.pin, (size_t)s.nbricks * 8, 0.0, s.stream))
    return bail(fail(SUSP_EDEVICE, "fill"));
  if (launch_fill_i32(s.cell_start, (size_t)s.ncell + 1, 0, s.stream)) return bail(fail(SUSP_EDEVICE, "fill"));
  // every node fluid and without links until k_links writes the records (it never runs
  // without spheres)
  if (launch_fill_i32((int32_t *)s.lrec, (size_t)s.nodes, 0, s.stream)) return bail(fail(SUSP_EDEVICE, "fill"));
  if (s.boundary == 1 && (launch_fill_f64(s.wacc, 8, 0.0, s.stream) || (n && launch_fill_f64(s.wfs, n * 3, 0.0, s.stream))))
    return bail(fail(SUSP_EDEVICE, "fill"));
  if (s.cbins > 0 && (launch_fill_f64(s.cacc, (size_t)(s.cbins + 1) * 6 + 8, 0.0, s.stream) ||
                      (n && launch_fill_i32(s.cflag, n * NCAP, 0, s.stream))))
    return bail(fail(SUSP_EDEVICE, "fill"));
  rc = remap(s);
  if (rc) return bail(rc);
  int32_t fl = 0;
  rc = read_flags(s, &fl);
  if (rc) return bail(rc);
  if (fl & 1) return bail(fail(SUSP_EUNSTABLE, "mapped spheres overlap in the initial state"));
  *out = h;
  return SUSP_OK;
}

extern "C" int susp_destroy(susp_sim *h) {
  if (!h) return SUSP_OK;
  for (int i = 0; i < PROF_EV * h->s.prof_cap; ++i) (void)hipEventDestroy(h->s.prof_ev[i]);
  free(h->s.prof_ev);
  (void)hipStreamSynchronize(h->s.stream);
  if (h->s.gexec) (void)hipGraphExecDestroy(h->s.gexec);
  free(h->s.clk_host);
  if (h->s.owns_block && h->s.block) (void)hipFree(h->s.block);
  delete h;
  return SUSP_OK;
}

// Protocol values of step t (shear offset and velocity at t and t+1, G', G'' weights).
static ClockEntry clock_entry(const Sim &s, int64_t t) {
  ClockEntry e;
  memset(&e, 0, sizeof e);
  protocol(s, t, &e.s, &e.ule);
  protocol(s, t + 1, &e.s1, &e.ule1);
  if (s.boundary == 1) { e.uw = wall_speed(s, t); e.uw1 = wall_speed(s, t + 1); }
  if (s.shear_kind == 2) {
    const int64_t tI = (int64_t)s.ncyc_I * s.period, tF = tI + (int64_t)s.ncyc_F * s.period;
    if (t >= tI && t < tF) {
      const double om = 2.0 * 3.14159265358979323846 / (double)s.period;
      const double ph = om * (double)(t - tI) + s.theta;
      e.gphase = 1;
      e.gcos = cos(ph);
      e.gsin = sin(ph);
    }
  }
  return e;
}

// Upload the protocol values of the next m <= CLK_CAP steps and rewind the device cursor.
// The staging table is reused by the next upload, hence the wait (for this stream only).
static int upload_clock(Sim &s, int m) {
  for (int k = 0; k < m; ++k) s.clk_host[k] = clock_entry(s, s.step + k);
  HIPCHK(hipMemcpyAsync(s.clk_tab, s.clk_host, (size_t)m * sizeof(ClockEntry), hipMemcpyHostToDevice, s.stream));
  HIPCHK(launch_clock(&s, 1));
  HIPCHK(hipStreamSynchronize(s.stream));
  return SUSP_OK;
}

// One lattice step (see the header for the order of the parts).  Every kernel argument is
// fixed except the buffer parities, which repeat every two steps; the shear offsets come
// from the device clock.
static int one_step(Sim &s) {
  const Box b = make_box(s, 0.0, 0.0);  // dimensions only
  HIPCHK(launch_clock(&s, 0));
  s.hcur ^= 1;
  if (s.n) {  // the pair search needs only the positions at the start of the step
    HIPCHK(launch_cells(&s, s.cell_start, s.cell_ids, s.cell_scr));
    HIPCHK(launch_pairs(&s, b));
    s.lcur ^= 1;
  }
  if (s.boundary == 1) HIPCHK(launch_walls(&s));
  else HIPCHK(launch_ghosts(&s, b, s.gown, s.gcnt, s.gval, 1, s.clk, 1));
  hipEvent_t *ev = nullptr;
  if (s.prof_on) {
    if (s.prof_used == s.prof_cap) {
      const int cap = s.prof_cap ? 2 * s.prof_cap : 256;
      hipEvent_t *nev = (hipEvent_t *)realloc(s.prof_ev, sizeof(hipEvent_t) * PROF_EV * cap);
      if (!nev) return fail(SUSP_ENOMEM, "event pool");
      for (int i = PROF_EV * s.prof_cap; i < PROF_EV * cap; ++i) HIPCHK(hipEventCreate(&nev[i]));
      s.prof_ev = nev;
      s.prof_cap = cap;
    }
    ev = &s.prof_ev[PROF_EV * s.prof_used++];
    HIPCHK(hipEventRecord(ev[0], s.stream));
  }
  HIPCHK(launch_links(&s, b));
  if (ev) HIPCHK(hipEventRecord(ev[1], s.stream));
  HIPCHK(launch_lbm(&s, b));
  if (ev) HIPCHK(hipEventRecord(ev[2], s.stream));
  s.cur ^= 1;
  if (s.n) {
    HIPCHK(launch_pair_rev(&s));
    for (int k = 0; k < s.n_sub; ++k) {
      HIPCHK(launch_substep(&s, b, k));
      s.pcur ^= 1;
    }
    s.hfin = (1 - s.hfin + s.n_sub) & 1;
    HIPCHK(launch_map_update(&s, b, 1));
    HIPCHK(launch_map_update(&s, b, 2));
  }
  if (s.boundary == 1) HIPCHK(launch_wall_force(&s));
  HIPCHK(launch_stress(&s));
  HIPCHK(launch_contact_sample(&s));
  s.step += 1;
  return SUSP_OK;
}

static int parity(const Sim &s) { return s.cur | (s.lcur << 1) | (s.hcur << 2) | (s.pcur << 3) | (s.hfin << 4); }

// Record 2 x graph_on steps on the simulation's stream as one graph.  The buffer parities
// repeat every two steps, so the graph replays from the parity it was recorded at;
// recording does not execute anything, so the host clock is restored afterwards.
static int record_graph(Sim &s) {
  const int64_t step = s.step;
  const int par = parity(s);
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal));
  int rc = SUSP_OK;
  for (int k = 0; k < 2 * s.graph_on && !rc; ++k) rc = one_step(s);
  hipError_t e = hipStreamEndCapture(s.stream, &g);
  s.step = step;
  if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
  if (e != hipSuccess) return fail(SUSP_EDEVICE, "graph capture: %s", hipGetErrorString(e));
  if (parity(s) != par) { (void)hipGraphDestroy(g); return fail(SUSP_ESTATE, "step parities do not repeat"); }
  e = hipGraphInstantiate(&s.gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) { s.gexec = nullptr; return fail(SUSP_EDEVICE, "graph instantiate: %s", hipGetErrorString(e)); }
  s.gparity = par;
  return SUSP_OK;
}

// m steps whose clock table is on the device: runs of 2 x graph_on steps by graph replay
// where possible.
static int run_steps(Sim &s, int m) {
  const bool graph = s.graph_on > 0 && s.stream != nullptr && !s.prof_on;
  const int gs = 2 * s.graph_on;
  int k = 0;
  if (graph && m >= gs) {
    if (!s.gexec) {
      int rc = record_graph(s);
      if (rc) return rc;
    }
    if (parity(s) != s.gparity) {  // one plain step brings the parities back
      int rc = one_step(s);
      if (rc) return rc;
      ++k;
    }
    for (; k + gs <= m; k += gs) {
      HIPCHK(hipGraphLaunch(s.gexec, s.stream));
      s.step += gs;
    }
  }
  for (; k < m; ++k) {
    int rc = one_step(s);
    if (rc) return rc;
  }
  return SUSP_OK;
}

namespace susp {

// ---- multi-job batches (batch.hip) ----
Sim &sim_of(susp_sim *h) { return h->s; }

// Whether the simulation's step can run in multi-job launches: every kernel of its step has
// a multi-job form (Lees-Edwards, spheres in the fused lattice kernel, explicit lubrication,
// no contact statistics, no profiling events), and two steps' launches (10 + n_sub each) fit
// the recorder.
bool multi_ok(const susp_sim *h) {
  const Sim &s = h->s;
  return s.boundary == 0 && s.n > 0 && s.BY == 4 && s.BZ == 4 && s.cbins == 0 && s.lub_implicit == 0 &&
         !s.prof_on && 2 * (10 + s.n_sub) <= 256;
}

// Record the launches of the next two steps into c without issuing them; the simulation's
// step counter and buffer parities are as before afterwards (they repeat every two steps).
int record_two_steps(susp_sim *h, Collect *c) {
  Sim &s = h->s;
  const int64_t step = s.step;
  const int par = parity(s);
  c->clear();
  s.col = c;
  int rc = one_step(s);
  if (!rc) rc = one_step(s);
  s.col = nullptr;
  s.step = step;
  if (rc) return rc;
  if (c->overflow) return fail(SUSP_ESTATE, "too many launches to record");
  if (parity(s) != par) return fail(SUSP_ESTATE, "step parities do not repeat");
  return SUSP_OK;
}

// Upload the protocol values of the next m <= CLK_CAP steps (waits for the simulation's
// stream), and count the steps as taken.
int prepare_run(susp_sim *h, int m) {
  if (m < 0 || m > CLK_CAP) return fail(SUSP_EINVAL, "run length out of range");
  int rc = upload_clock(h->s, m);
  return rc;
}
void advance_steps(susp_sim *h, int m) { h->s.step += m; }
int step_parity(const susp_sim *h) { return parity(h->s); }

// Queue nsteps steps on the simulation's stream (clock uploads wait only for their own copy).
int launch_steps(susp_sim *h, int64_t nsteps) {
  if (!h) return fail(SUSP_EINVAL, "NULL simulation");
  if (nsteps < 0) return fail(SUSP_EINVAL, "negative step count");
  Sim &s = h->s;
  for (int64_t done = 0; done < nsteps;) {
    const int m = (int)(nsteps - done < CLK_CAP ? nsteps - done : CLK_CAP);
    int rc = upload_clock(s, m);
    if (!rc) rc = run_steps(s, m);
    if (rc) return rc;
    done += m;
  }
  return SUSP_OK;
}

// Wait for the simulation's stream and turn its instability flags into a status.
int check_flags(susp_sim *h) {
  int32_t fl = 0;
  int rc = read_flags(h->s, &fl);
  if (rc) return rc;
  if (fl) {
    return fail(SUSP_EUNSTABLE, "instability flags 0x%x (1 mapped overlap, 2 non-finite particle state, "
                "4 neighbour overflow, 8 node touching more than six spheres, 16 sphere moved more than "
                "a node in a step, 32 fluid density or velocity not finite, 64 fluid mass plus "
                "ledger drifted)", fl);
  }
  return SUSP_OK;
}

int set_error(int code, const char *msg) { return fail(code, "%s", msg); }

}  // namespace susp

extern "C" int susp_step(susp_sim *h, int64_t nsteps) {
  int rc = launch_steps(h, nsteps);
  return rc ? rc : check_flags(h);
}

extern "C" int susp_stress(susp_sim *h, double out[5][6], double gg[2]) {
  if (!h || !out || !gg) return fail(SUSP_EINVAL, "NULL argument");
  Sim &s = h->s;
  double acc[65];
  HIPCHK(hipMemcpyAsync(acc, s.acc, sizeof acc, hipMemcpyDeviceToHost, s.stream));
  HIPCHK(hipStreamSynchronize(s.stream));
  const double n = acc[60] > 0 ? acc[60] : 1.0;
  for (int k = 0; k < 5; ++k)
    for (int c = 0; c < 6; ++c) out[k][c] = acc[30 + 6 * k + c] / n;
  if (acc[63] > 0 && s.g0_F != 0.0) {
    const double cf = 2.0 / (acc[63] * s.g0_F);
    gg[0] = -cf * acc[61];
    gg[1] = cf * acc[62];
  } else {
    gg[0] = 0.0;
    gg[1] = 0.0;
  }
  HIPCHK(launch_fill_f64(s.acc + 30, 31, 0.0, s.stream));
  HIPCHK(hipStreamSynchronize(s.stream));
  return SUSP_OK;
}

extern "C" int susp_health(susp_sim *h, double out[3]) {
  if (!h || !out) return fail(SUSP_EINVAL, "NULL argument");
  Sim &s = h->s;
  int32_t w[4];
  double a[5];
  HIPCHK(hipMemcpyAsync(w, s.flags + FL_HEALTH, sizeof w, hipMemcpyDeviceToHost, s.stream));
  HIPCHK(hipMemcpyAsync(a, s.acc + 64, sizeof a, hipMemcpyDeviceToHost, s.stream));
  HIPCHK(hipStreamSynchronize(s.stream));
  uint64_t nfast;
  memcpy(&nfast, w, 8);
  float umax2;
  memcpy(&umax2, &w[2], 4);
  out[0] = (double)nfast;
  out[1] = sqrt((double)umax2 * 3.0);  // |u| / c_s, c_s^2 = 1/3
  // fluid mass of the last step a[1] with the ledger before that step's covers a[4], against
  // the reference a[2] (taken at the first step after creation or a state load, a[3] = 1)
  out[2] = a[3] != 0.0 && a[2] > 0 ? fabs(a[1] + a[4] - a[2]) / a[2] : 0.0;
  HIPCHK(launch_fill_i32(s.flags + FL_HEALTH, 4, 0, s.stream));
  HIPCHK(hipStreamSynchronize(s.stream));
  return SUSP_OK;
}

extern "C" int susp_wall_force(susp_sim *h, double out[6]) {
  if (!h || !out) return fail(SUSP_EINVAL, "NULL argument");
  Sim &s = h->s;
  if (s.boundary != 1) return fail(SUSP_EINVAL, "no walls (boundary = 0)");
  double w[8];
  HIPCHK(hipMemcpyAsync(w, s.wacc, sizeof w, hipMemcpyDeviceToHost, s.stream));
  HIPCHK(hipStreamSynchronize(s.stream));
  const double n = w[6] > 0 ? w[6] : 1.0;
  for (int c = 0; c < 6; ++c) out[c] = w[c] / n;
  HIPCHK(launch_fill_f64(s.wacc, 8, 0.0, s.stream));
  HIPCHK(hipStreamSynchronize(s.stream));
  return SUSP_OK;
}

extern "C" int susp_contact_stats(susp_sim *h, int32_t nbins, double *hist, double summary[12]) {
  if (!h || !hist || !summary) return fail(SUSP_EINVAL, "NULL argument");
  Sim &s = h->s;
  if (s.cbins <= 0) return fail(SUSP_EINVAL, "contact statistics are off (contact_bins = 0)");
  if (nbins != s.cbins) return fail(SUSP_EINVAL, "nbins %d differs from contact_bins %d", nbins, s.cbins);
  HIPCHK(launch_contact_final(&s, s.cout));
  HIPCHK(hipMemcpyAsync(hist, s.cout, (size_t)5 * nbins * 8, hipMemcpyDeviceToHost, s.stream));
  HIPCHK(hipMemcpyAsync(summary, s.cout + (size_t)5 * nbins, 12 * 8, hipMemcpyDeviceToHost, s.stream));
  HIPCHK(hipStreamSynchronize(s.stream));
  return SUSP_OK;
}

// ---------------------------------------------------------------------------------------
// The contact read-out for callers that cannot allocate: the final kernel's staging (the
// per-bin results and the summary) is a static device array instead of the simulation's
// own.  Each device holds one copy for the life of the process; its address comes from
// hipGetSymbolAddress once per device, with that device current, and only that address
// (never the array's name, a host-side stand-in) reaches kernels and copies.  Calls are
// serialised by the lock below, so calls from several host threads do not overlap on the
// array; the kernel writes every element it hands back, so nothing is cleared first.
constexpr int NOALLOC_BINS = 180;  // largest bin count the static staging holds (1 degree)
static __device__ __align__(256) double scratch[5 * NOALLOC_BINS + 12];
static std::mutex scratch_mu;
static std::map<int, double *> scratch_ptr;  // device -> device address of scratch

// Device address of the staging on device dev (scratch_mu held).
static int scratch_on(int dev, double **out) {
  auto it = scratch_ptr.find(dev);
  if (it != scratch_ptr.end()) {
    *out = it->second;
    return SUSP_OK;
  }
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(SUSP_EDEVICE, "hipGetDevice");
  if (cur != dev && hipSetDevice(dev) != hipSuccess) return fail(SUSP_EDEVICE, "hipSetDevice(%d)", dev);
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != dev) (void)hipSetDevice(cur);
  if (e != hipSuccess || !p)
    return fail(SUSP_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
  scratch_ptr[dev] = (double *)p;
  *out = (double *)p;
  return SUSP_OK;
}

extern "C" int susp_contact_stats_noalloc(susp_sim *h, int32_t nbins, double *hist, double summary[12]) {
  if (!h || !hist || !summary) return fail(SUSP_EINVAL, "NULL argument");
  Sim &s = h->s;
  if (s.cbins <= 0) return fail(SUSP_EINVAL, "contact statistics are off (contact_bins = 0)");
  if (nbins != s.cbins) return fail(SUSP_EINVAL, "nbins %d differs from contact_bins %d", nbins, s.cbins);
  if (nbins > NOALLOC_BINS)
    return fail(SUSP_EINVAL, "nbins %d is above the %d bins of the static staging", nbins, NOALLOC_BINS);
  std::lock_guard<std::mutex> lock(scratch_mu);
  double *stage = nullptr;
  const int rc = scratch_on(s.device, &stage);
  if (rc) return rc;
  HIPCHK(launch_contact_final(&s, stage));
  HIPCHK(hipMemcpyAsync(hist, stage, (size_t)5 * nbins * 8, hipMemcpyDeviceToHost, s.stream));
  HIPCHK(hipMemcpyAsync(summary, stage + (size_t)5 * nbins, 12 * 8, hipMemcpyDeviceToHost, s.stream));
  HIPCHK(hipStreamSynchronize(s.stream));
  return SUSP_OK;
}

// ---------------------------------------------------------------------------------------
// The spare population buffer (the one the next step writes) stages FP64 values one plane
// at a time: 19 planes of the storage type hold at least one FP64 plane plus its padding, so
// no device memory is allocated (a batch's other jobs never wait for an allocation).
extern "C" int susp_get_populations(susp_sim *h, double *host) {
  if (!h || !host) return fail(SUSP_EINVAL, "NULL argument");
  Sim &s = h->s;
  double *stage = (double *)s.f[1 - s.cur];
  for (int q = 0; q < NQ; ++q) {
    HIPCHK(launch_pop_plane(&s, stage, q, 0));
    HIPCHK(hipMemcpyAsync(host + (size_t)q * s.nodes, stage, (size_t)s.nodes * 8, hipMemcpyDeviceToHost, s.stream));
  }
  HIPCHK(hipStreamSynchronize(s.stream));
  return SUSP_OK;
}

extern "C" int susp_set_populations(susp_sim *h, const double *host) {
  if (!h || !host) return fail(SUSP_EINVAL, "NULL argument");
  Sim &s = h->s;
  double *stage = (double *)s.f[1 - s.cur];
  HIPCHK(hipStreamSynchronize(s.stream));
  for (int q = 0; q < NQ; ++q) {
    HIPCHK(hipMemcpyAsync(stage, host + (size_t)q * s.nodes, (size_t)s.nodes * 8, hipMemcpyHostToDevice, s.stream));
    HIPCHK(launch_pop_plane(&s, stage, q, 1));
  }
  int rc = reset_mass_reference(s);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(s.stream));
  return SUSP_OK;
}

// ---- whole-state checkpoint: header, populations as stored, particles, history, running sums
namespace {
struct StateHeader {
  char magic[8];  // "SUSPSTA1"
  int32_t precision, lx, ly, lz, n, npairs;
  int64_t step;
  int64_t nodes, es;  // nodes and bytes per stored population element
};
// bytes of the stored populations, padded so that the FP64 parts after them stay aligned
size_t state_pop_bytes(const Sim &s) {
  const size_t es = s.precision == 0 ? 8 : s.precision == 1 ? 4 : 2;
  return ((size_t)NQ * s.nodes * es + 7) / 8 * 8;
}
size_t state_bytes(const Sim &s, int npairs) {
  return sizeof(StateHeader) + state_pop_bytes(s) + (size_t)s.n * 13 * 8 + (size_t)npairs * (8 + 24) +
         (size_t)SUSP_NACC * 8;
}
}  // namespace

extern "C" int susp_get_state(susp_sim *h, void *host, size_t *bytes) {
  if (!h || !bytes) return fail(SUSP_EINVAL, "NULL argument");
  Sim &s = h->s;
  int32_t np = 0;
  int rc = susp_get_history(h, 0, &np, nullptr, nullptr, nullptr);
  if (rc) return rc;
  const size_t need = state_bytes(s, np);
  if (!host) {
    *bytes = need;
    return SUSP_OK;
  }
  if (*bytes < need) return fail(SUSP_EINVAL, "state buffer of %zu bytes, %zu needed", *bytes, need);
  char *p = (char *)host;
  StateHeader hd;
  memset(&hd, 0, sizeof hd);
  memcpy(hd.magic, "SUSPSTA1", 8);
  hd.precision = s.precision; hd.lx = s.lx; hd.ly = s.ly; hd.lz = s.lz; hd.n = s.n; hd.npairs = np;
  hd.step = s.step;
  hd.nodes = s.nodes;
  hd.es = s.precision == 0 ? 8 : s.precision == 1 ? 4 : 2;
  memcpy(p, &hd, sizeof hd);
  p += sizeof hd;
  // the populations exactly as stored (deviations from the rest state in the storage type)
  HIPCHK(hipStreamSynchronize(s.stream));
  memset(p, 0, state_pop_bytes(s));
  for (int q = 0; q < NQ; ++q)
    HIPCHK(hipMemcpy(p + (size_t)q * s.nodes * hd.es, (const char *)s.f[s.cur] + (size_t)q * s.plane * hd.es,
                     (size_t)s.nodes * hd.es, hipMemcpyDeviceToHost));
  p += state_pop_bytes(s);
  double *d = (double *)p;
  rc = susp_get_particles(h, d, d + 3 * (size_t)s.n, d + 6 * (size_t)s.n, d + 9 * (size_t)s.n);
  if (rc) return rc;
  p += (size_t)s.n * 13 * 8;
  int32_t got = 0;
  std::vector<int32_t> pi(np > 0 ? np : 1), pj(np > 0 ? np : 1);
  rc = susp_get_history(h, np, &got, pi.data(), pj.data(), (double *)(p + (size_t)np * 8));
  if (rc) return rc;
  if (got != np) return fail(SUSP_ESTATE, "spring history changed while it was read");
  memcpy(p, pi.data(), (size_t)np * 4);
  memcpy(p + (size_t)np * 4, pj.data(), (size_t)np * 4);
  p += (size_t)np * (8 + 24);
  rc = susp_get_accumulators(h, (double *)p);
  if (rc) return rc;
  *bytes = need;
  return SUSP_OK;
}

extern "C" int susp_set_state(susp_sim *h, const void *host, size_t bytes) {
  if (!h || !host) return fail(SUSP_EINVAL, "NULL argument");
  Sim &s = h->s;
  StateHeader hd;
  if (bytes < sizeof hd) return fail(SUSP_ESTATE, "state buffer too short");
  memcpy(&hd, host, sizeof hd);
  if (memcmp(hd.magic, "SUSPSTA1", 8) != 0) return fail(SUSP_ESTATE, "not a state buffer");
  if (hd.precision != s.precision || hd.lx != s.lx || hd.ly != s.ly || hd.lz != s.lz || hd.n != s.n ||
      hd.nodes != s.nodes || hd.npairs < 0)
    return fail(SUSP_ESTATE, "state of another simulation (precision, box or sphere count differ)");
  if (bytes != state_bytes(s, hd.npairs)) return fail(SUSP_ESTATE, "state buffer has the wrong size");
  const char *p = (const char *)host + sizeof hd;
  const char *pop = p;
  p += state_pop_bytes(s);
  const double *d = (const double *)p;
  int rc = susp_set_clock(h, hd.step);
  if (!rc) rc = susp_set_particles(h, d, d + 3 * (size_t)s.n, d + 6 * (size_t)s.n, d + 9 * (size_t)s.n);
  if (rc) return rc;
  p += (size_t)s.n * 13 * 8;
  HIPCHK(hipStreamSynchronize(s.stream));
  for (int q = 0; q < NQ; ++q)
    HIPCHK(hipMemcpy((char *)s.f[s.cur] + (size_t)q * s.plane * hd.es, pop + (size_t)q * s.nodes * hd.es,
                     (size_t)s.nodes * hd.es, hipMemcpyHostToDevice));
  rc = reset_mass_reference(s);
  if (rc) return rc;
  std::vector<int32_t> pi(hd.npairs > 0 ? hd.npairs : 1), pj(hd.npairs > 0 ? hd.npairs : 1);
  memcpy(pi.data(), p, (size_t)hd.npairs * 4);
  memcpy(pj.data(), p + (size_t)hd.npairs * 4, (size_t)hd.npairs * 4);
  rc = susp_set_history(h, hd.npairs, pi.data(), pj.data(), (const double *)(p + (size_t)hd.npairs * 8));
  if (rc) return rc;
  p += (size_t)hd.npairs * (8 + 24);
  return susp_set_accumulators(h, (const double *)p);
}

// acc layout on the device: [0,30) stress of the last step, [30,60) stress sums, 60 their
// count, 61 sum sigma_xy cos, 62 sum sigma_xy sin, 63 observation steps, 64 mass ledger
extern "C" int susp_get_accumulators(susp_sim *h, double out[SUSP_NACC]) {
  if (!h || !out) return fail(SUSP_EINVAL, "NULL argument");
  Sim &s = h->s;
  HIPCHK(hipMemcpyAsync(out, s.acc + 30, SUSP_NACC * 8, hipMemcpyDeviceToHost, s.stream));
  HIPCHK(hipStreamSynchronize(s.stream));
  return SUSP_OK;
}

extern "C" int susp_set_accumulators(susp_sim *h, const double in[SUSP_NACC]) {
  if (!h || !in) return fail(SUSP_EINVAL, "NULL argument");
  Sim &s = h->s;
  for (int k = 0; k < SUSP_NACC; ++k)
    if (!isfinite(in[k])) return fail(SUSP_EINVAL, "accumulator %d is not finite", k);
  if (in[30] < 0 || in[33] < 0) return fail(SUSP_EINVAL, "negative step counts");
  HIPCHK(hipStreamSynchronize(s.stream));
  HIPCHK(hipMemcpy(s.acc + 30, in, SUSP_NACC * 8, hipMemcpyHostToDevice));
  int rc = reset_mass_reference(s);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(s.stream));
  return SUSP_OK;
}

extern "C" int susp_get_particles(susp_sim *h, double *pos, double *vel, double *omega, double *quat) {
  if (!h) return fail(SUSP_EINVAL, "NULL simulation");
  Sim &s = h->s;
  const size_t n = (size_t)s.n;
  if (!n) return SUSP_OK;
  if (pos) HIPCHK(hipMemcpyAsync(pos, s.R[s.pcur], n * 24, hipMemcpyDeviceToHost, s.stream));
  if (vel) HIPCHK(hipMemcpyAsync(vel, s.U[s.pcur], n * 24, hipMemcpyDeviceToHost, s.stream));
  if (omega) HIPCHK(hipMemcpyAsync(omega, s.W[s.pcur], n * 24, hipMemcpyDeviceToHost, s.stream));
  if (quat) HIPCHK(hipMemcpyAsync(quat, s.Q[s.pcur], n * 32, hipMemcpyDeviceToHost, s.stream));
  HIPCHK(hipStreamSynchronize(s.stream));
  return SUSP_OK;
}

extern "C" int susp_set_particles(susp_sim *h, const double *pos, const double *vel,
                                  const double *omega, const double *quat) {
  if (!h) return fail(SUSP_EINVAL, "NULL simulation");
  Sim &s = h->s;
  const size_t n = (size_t)s.n;
  if (!n) return SUSP_OK;
  if (pos)
    for (size_t i = 0; i < n; ++i)
      for (int c = 0; c < 3; ++c) {
        const double L = c == 0 ? s.lx : (c == 1 ? s.ly : s.lz);
        if (!(pos[3 * i + c] >= 0.0 && pos[3 * i + c] < L)) return fail(SUSP_EINVAL, "sphere %zu outside the box", i);
      }
  HIPCHK(hipStreamSynchronize(s.stream));
  if (pos) HIPCHK(hipMemcpy(s.R[s.pcur], pos, n * 24, hipMemcpyHostToDevice));
  if (vel) HIPCHK(hipMemcpy(s.U[s.pcur], vel, n * 24, hipMemcpyHostToDevice));
  if (omega) HIPCHK(hipMemcpy(s.W[s.pcur], omega, n * 24, hipMemcpyHostToDevice));
  if (quat) HIPCHK(hipMemcpy(s.Q[s.pcur], quat, n * 32, hipMemcpyHostToDevice));
  int rc = remap(s);
  if (rc) return rc;
  int32_t fl = 0;
  rc = read_flags(s, &fl);
  if (rc) return rc;
  if (fl & 1) return fail(SUSP_EUNSTABLE, "mapped spheres overlap");
  return SUSP_OK;
}

extern "C" int susp_get_history(susp_sim *h, int32_t cap, int32_t *count, int32_t *oi, int32_t *oj,
                                double *xi) {
  if (!h || !count) return fail(SUSP_EINVAL, "NULL argument");
  Sim &s = h->s;
  const size_t n = (size_t)s.n;
  *count = 0;
  if (!n) return SUSP_OK;
  std::vector<int32_t> cnt(n), nj(n * NCAP), on(n * NCAP);
  std::vector<double> hx(n * NCAP * 3);
  HIPCHK(hipMemcpyAsync(cnt.data(), s.ncnt[s.lcur], n * 4, hipMemcpyDeviceToHost, s.stream));
  HIPCHK(hipMemcpyAsync(nj.data(), s.nj[s.lcur], n * NCAP * 4, hipMemcpyDeviceToHost, s.stream));
  HIPCHK(hipMemcpyAsync(on.data(), s.hon[s.hfin], n * NCAP * 4, hipMemcpyDeviceToHost, s.stream));
  HIPCHK(hipMemcpyAsync(hx.data(), s.hxi[s.hfin], n * NCAP * 24, hipMemcpyDeviceToHost, s.stream));
  HIPCHK(hipStreamSynchronize(s.stream));
  int32_t k = 0;
  for (size_t i = 0; i < n; ++i)
    for (int u = 0; u < cnt[i]; ++u) {
      const size_t e = i * NCAP + u;
      if (nj[e] <= (int32_t)i || !on[e]) continue;
      if (oi && k < cap) {
        oi[k] = (int32_t)i;
        if (oj) oj[k] = nj[e];
        if (xi) { xi[3 * k] = hx[3 * e]; xi[3 * k + 1] = hx[3 * e + 1]; xi[3 * k + 2] = hx[3 * e + 2]; }
      }
      ++k;
    }
  *count = k;
  return SUSP_OK;
}

extern "C" int susp_set_history(susp_sim *h, int32_t count, const int32_t *hi, const int32_t *hj,
                                const double *xi) {
  if (!h || count < 0 || (count > 0 && (!hi || !hj || !xi))) return fail(SUSP_EINVAL, "bad arguments");
  Sim &s = h->s;
  const size_t n = (size_t)s.n;
  if (!n) return count ? fail(SUSP_EINVAL, "no spheres") : SUSP_OK;
  std::vector<int32_t> cnt(n, 0), nj(n * NCAP, 0), on(n * NCAP, 0);
  std::vector<double> hx(n * NCAP * 3, 0.0);
  for (int32_t k = 0; k < count; ++k) {
    const int32_t i = hi[k], j = hj[k];
    if (i < 0 || j <= i || j >= (int32_t)n) return fail(SUSP_EINVAL, "history pair %d invalid", k);
    if (cnt[i] >= NCAP) return fail(SUSP_EINVAL, "too many history pairs for sphere %d", i);
    const size_t e = (size_t)i * NCAP + cnt[i]++;
    nj[e] = j;
    on[e] = 1;
    hx[3 * e] = xi[3 * k]; hx[3 * e + 1] = xi[3 * k + 1]; hx[3 * e + 2] = xi[3 * k + 2];
  }
  HIPCHK(hipStreamSynchronize(s.stream));
  HIPCHK(hipMemcpy(s.ncnt[s.lcur], cnt.data(), n * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(s.nj[s.lcur], nj.data(), n * NCAP * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(s.hon[s.hfin], on.data(), n * NCAP * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(s.hxi[s.hfin], hx.data(), n * NCAP * 24, hipMemcpyHostToDevice));
  return SUSP_OK;
}

extern "C" int susp_get_clock(susp_sim *h, int64_t *step, double *offset) {
  if (!h) return fail(SUSP_EINVAL, "NULL simulation");
  double off, ule;
  protocol(h->s, h->s.step, &off, &ule);
  if (step) *step = h->s.step;
  if (offset) *offset = off;
  return SUSP_OK;
}

extern "C" int susp_set_clock(susp_sim *h, int64_t step) {
  if (!h || step < 0) return fail(SUSP_EINVAL, "bad arguments");
  HIPCHK(hipStreamSynchronize(h->s.stream));
  h->s.step = step;
  // re-map with the offset of the new clock; overlaps are reported by the next
  // susp_set_particles or susp_step (positions are usually replaced right after)
  int rc = remap(h->s);
  if (rc) return rc;
  int32_t fl = 0;
  return read_flags(h->s, &fl);
}

extern "C" int susp_get_hydro(susp_sim *h, double *force, double *torque, double *stresslet,
                              int32_t *nlinks) {
  if (!h) return fail(SUSP_EINVAL, "NULL simulation");
  Sim &s = h->s;
  const size_t n = (size_t)s.n;
  if (!n) return SUSP_OK;
  std::vector<double> v(n * HYD);
  HIPCHK(hipMemcpyAsync(v.data(), s.hyd[s.hcur], n * HYD * 8, hipMemcpyDeviceToHost, s.stream));
  HIPCHK(hipStreamSynchronize(s.stream));
  for (size_t i = 0; i < n; ++i) {
    const double *a = &v[i * HYD];
    for (int c = 0; c < 3; ++c) {
      if (force) force[3 * i + c] = a[c];
      if (torque) torque[3 * i + c] = a[3 + c];
    }
    for (int c = 0; c < 6; ++c)
      if (stresslet) stresslet[6 * i + c] = a[6 + c];
    if (nlinks) nlinks[i] = (int32_t)llround(a[12]);
  }
  return SUSP_OK;
}

extern "C" int susp_get_derived(susp_sim *h, double out[10]) {
  if (!h || !out) return fail(SUSP_EINVAL, "NULL argument");
  const Sim &s = h->s;
  const double v[10] = {s.m0, s.kn, s.kt, s.eta_n, s.lub_delta, s.F0, s.lambda, s.eta0, s.a_min, s.a_max};
  memcpy(out, v, sizeof v);
  return SUSP_OK;
}

extern "C" int susp_get_lists(susp_sim *h, int32_t kind, void *host, size_t *bytes) {
  if (!h || !bytes) return fail(SUSP_EINVAL, "NULL argument");
  Sim &s = h->s;
  const size_t n = (size_t)s.n;
  std::vector<int32_t> out;
  HIPCHK(hipStreamSynchronize(s.stream));
  if (kind == SUSP_LIST_OWNER) {
    out.resize((size_t)s.nodes);
    HIPCHK(hipMemcpy(out.data(), s.own, out.size() * 4, hipMemcpyDeviceToHost));
  } else if (kind == SUSP_LIST_GHOST) {
    out.resize((size_t)2 * s.lx * s.lz);
    HIPCHK(hipMemcpy(out.data(), s.gown, out.size() * 4, hipMemcpyDeviceToHost));
  } else if (kind == SUSP_LIST_CELLS) {
    out.resize((size_t)s.ncell + 1 + n);
    HIPCHK(hipMemcpy(out.data(), s.cell_start, ((size_t)s.ncell + 1) * 4, hipMemcpyDeviceToHost));
    if (n) HIPCHK(hipMemcpy(out.data() + s.ncell + 1, s.cell_ids, n * 4, hipMemcpyDeviceToHost));
  } else if (kind == SUSP_LIST_PAIRS || kind == SUSP_LIST_CONTACTS) {
    if (n) {
      std::vector<int32_t> cnt(n), nj(n * NCAP), hs(n * NCAP);
      HIPCHK(hipMemcpy(cnt.data(), s.ncnt[s.lcur], n * 4, hipMemcpyDeviceToHost));
      HIPCHK(hipMemcpy(nj.data(), s.nj[s.lcur], n * NCAP * 4, hipMemcpyDeviceToHost));
      HIPCHK(hipMemcpy(hs.data(), s.hstart, n * NCAP * 4, hipMemcpyDeviceToHost));
      for (size_t i = 0; i < n; ++i)
        for (int u = 0; u < cnt[i] && u < NCAP; ++u) {
          const size_t e = i * NCAP + u;
          if (nj[e] <= (int32_t)i) continue;
          if (kind == SUSP_LIST_CONTACTS && !hs[e]) continue;
          out.push_back((int32_t)i);
          out.push_back(nj[e]);
        }
    }
  } else if (kind == SUSP_LIST_LINKS) {
    // staged through the spare population buffer: the ghost owners of the current offset
    // after one plane of link owners (the buffer holds far more than nodes + 2 lx lz words)
    double off, ule;
    protocol(s, s.step, &off, &ule);
    const Box b = make_box(s, off, ule);
    int32_t *lk = (int32_t *)s.f[1 - s.cur];
    int32_t *g = lk + ((size_t)s.nodes + 63) / 64 * 64;
    if (n) HIPCHK(launch_cells(&s, s.cell_start, s.cell_ids, s.cell_scr));
    HIPCHK(n && s.boundary == 0 ? launch_ghosts(&s, b, g, g + 2 * (size_t)s.lx * s.lz, s.gval, 0, nullptr, 0)
                                : launch_fill_i32(g, (size_t)2 * s.lx * s.lz, -1, s.stream));
    std::vector<int32_t> all((size_t)NQ * s.nodes, -1);
    for (int q = 1; q < NQ; ++q) {
      HIPCHK(launch_link_enum(&s, g, lk, q));
      HIPCHK(hipMemcpyAsync(all.data() + (size_t)q * s.nodes, lk, (size_t)s.nodes * 4, hipMemcpyDeviceToHost, s.stream));
    }
    HIPCHK(hipStreamSynchronize(s.stream));
    for (int64_t node = 0; node < s.nodes; ++node)
      for (int q = 1; q < NQ; ++q) {
        const int32_t o = all[(size_t)q * s.nodes + node];
        if (o >= 0) { out.push_back((int32_t)node); out.push_back(q); out.push_back(o); }
      }
  } else {
    return fail(SUSP_EINVAL, "unknown list kind %d", kind);
  }
  const size_t need = out.size() * 4;
  const size_t cap = *bytes;
  *bytes = need;
  if (host) {
    if (cap < need) return fail(SUSP_EINVAL, "buffer of %zu bytes < %zu", cap, need);
    memcpy(host, out.data(), need);
  }
  return SUSP_OK;
}

extern "C" int susp_use_graphs(susp_sim *h, int32_t pairs) {
  if (!h) return fail(SUSP_EINVAL, "NULL simulation");
  if (pairs < 0 || pairs > 64) return fail(SUSP_EINVAL, "pairs must be in [0, 64]");
  if (pairs != h->s.graph_on && h->s.gexec) {
    HIPCHK(hipStreamSynchronize(h->s.stream));
    (void)hipGraphExecDestroy(h->s.gexec);
    h->s.gexec = nullptr;
  }
  h->s.graph_on = pairs;
  return SUSP_OK;
}

extern "C" int susp_profile(susp_sim *h, int32_t enable) {
  if (!h) return fail(SUSP_EINVAL, "NULL simulation");
  h->s.prof_on = enable ? 1 : 0;
  return SUSP_OK;
}

extern "C" int susp_profile_read(susp_sim *h, double *ms_total, int64_t *launches) {
  double parts[2];
  int rc = susp_profile_read_parts(h, parts, launches);
  if (rc == SUSP_OK && ms_total) *ms_total = parts[1];
  return rc;
}

extern "C" int susp_profile_read_parts(susp_sim *h, double ms[2], int64_t *launches) {
  if (!h || !ms || !launches) return fail(SUSP_EINVAL, "NULL argument");
  Sim &s = h->s;
  HIPCHK(hipStreamSynchronize(s.stream));
  double tot[2] = {0.0, 0.0};
  for (int i = 0; i < s.prof_used; ++i) {
    for (int k = 0; k < 2; ++k) {
      float t = 0.0f;
      HIPCHK(hipEventElapsedTime(&t, s.prof_ev[PROF_EV * i + k], s.prof_ev[PROF_EV * i + k + 1]));
      tot[k] += t;
    }
  }
  ms[0] = tot[0];
  ms[1] = tot[1];
  *launches = s.prof_used;
  s.prof_used = 0;
  return SUSP_OK;
}
