/*
 * susp_oracle.c -- plain FP64 CPU reference of the sheared-suspension LBM + DEM step.
 *
 * TEST INFRASTRUCTURE ONLY: the GPU library never includes, links or calls this file.
 * It is written for a reader checking it against Pradipto & Hayakawa (arXiv:1904.02929):
 *   equations of motion             eq. (1)
 *   contact force / torque           eqs. (11), (11t) and the spring-dashpot text of Sec. 2
 *   contact / DLVO stress            eqs. (12), (14)
 *   DLVO repulsion                   eq. (13)
 *   total stress                     eq. (15)
 *   oscillatory strain, G', G''      eqs. (16)-(18)
 *   contact statistics               eqs. (19)-(23), (26)-(27), App. C; Delta lambda / P
 *   LB update, moments, collision    App. A eqs. (3)-(5): single-time BGK, or the linearised
 *                                    operator of eq. (5) with separate eigenvalues for the
 *                                    shear stress, its trace and the ghost modes
 *   moving bounce-back, link force   App. A eqs. (6)-(8); force and torque sums eqs. (9)-(10)
 *   mapped radius, lubrication       App. A (mapped radius 0.95 a; grand-resistance matrix
 *                                    with the leading-order scalar functions)
 * The Lees-Edwards boundary is not in the paper; it follows the interpolated, Galilean
 * corrected ghost-row scheme of Wagner & Pagonabarraga (2002).
 * Compile with -ffp-contract=off: every geometric predicate is evaluated left to right.
 */
#include "susp_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------- D3Q19 lattice (App. A: weights 1/3, 1/18, 1/36) ---------------- */
static const int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
static double WQ(int q) { return q == 0 ? 1.0 / 3.0 : (q <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }
static int OPP(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }
/* directions entering row y=0 from below (c_y=+1) and row y=ly-1 from above (c_y=-1) */
static const int UPQ[5] = {3, 7, 10, 15, 17};
static const int DNQ[5] = {4, 8, 9, 16, 18};

void orc_lattice(int32_t *cx, int32_t *cy, int32_t *cz, double *w, int32_t *opp) {
  for (int q = 0; q < 19; ++q) {
    cx[q] = CX[q]; cy[q] = CY[q]; cz[q] = CZ[q]; w[q] = WQ(q); opp[q] = OPP(q);
  }
}

static const double PI = 3.14159265358979323846;

/* Second-order equilibrium (the standard D3Q19 form; the paper defers to Succi). */
void orc_feq(double rho, double ux, double uy, double uz, double out[19]) {
  double uu = ux * ux + uy * uy + uz * uz;
  for (int q = 0; q < 19; ++q) {
    double cu = CX[q] * ux + CY[q] * uy + CZ[q] * uz;
    out[q] = WQ(q) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
}
static double feq1(int q, double rho, double ux, double uy, double uz) {
  double uu = ux * ux + uy * uy + uz * uz;
  double cu = CX[q] * ux + CY[q] * uy + CZ[q] * uz;
  return WQ(q) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}

/* ---------------- geometry ---------------- */
/* Minimum-image displacement d = point - particle under Lees-Edwards in y (offset s) and
 * periodicity in x, z.  k is the image index of the particle: the image sits at
 * R + k (s, ly, 0) and moves with U + k U_LE x.                                          */
void orc_minimage(const orc_params *p, double s, double dx, double dy, double dz,
                  double out[3], int32_t *k) {
  double Lx = p->lx, Ly = p->ly, Lz = p->lz;
  int kk = 0;
  if (dy > 0.5 * Ly) { dy -= Ly; dx -= s; kk = 1; }
  else if (dy < -0.5 * Ly) { dy += Ly; dx += s; kk = -1; }
  for (int it = 0; it < 4 && dx > 0.5 * Lx; ++it) dx -= Lx;
  for (int it = 0; it < 4 && dx < -0.5 * Lx; ++it) dx += Lx;
  for (int it = 0; it < 4 && dz > 0.5 * Lz; ++it) dz -= Lz;
  for (int it = 0; it < 4 && dz < -0.5 * Lz; ++it) dz += Lz;
  out[0] = dx; out[1] = dy; out[2] = dz;
  if (k) *k = kk;
}

static int wrapi(int i, int L) { i %= L; return i < 0 ? i + L : i; }

/* ---------------- shear protocol: eq. (16) and its rate ---------------- */
static void le_protocol(const orc_params *p, int64_t t, double *s, double *ule) {
  double Lx = p->lx, Ly = p->ly;
  if (p->shear_kind == 1) {
    double u = p->gamma_dot * Ly;
    double x = (double)t * u;
    *s = x - Lx * floor(x / Lx);
    *ule = u;
  } else if (p->shear_kind == 2) {
    int64_t P = p->period;
    int64_t tI = (int64_t)p->ncyc_I * P;
    double g0 = t < tI ? p->g0_I : p->g0_F;
    int64_t tp = t < tI ? t : t - tI;
    double om = 2.0 * PI / (double)P;
    double ph = om * (double)tp + p->theta;
    double gam = g0 * (cos(p->theta) - cos(ph));
    double gdot = om * g0 * sin(ph);
    double x = Ly * gam;
    *s = x - Lx * floor(x / Lx);
    *ule = Ly * gdot;
  } else {
    *s = 0.0; *ule = 0.0;
  }
}

/* Lees-Edwards offset and sliding velocity at step t; with walls there is no sliding plane */
void orc_protocol(const orc_params *p, int64_t t, double *s, double *ule) {
  if (p->boundary == 1) { *s = 0.0; *ule = 0.0; return; }
  le_protocol(p, t, s, ule);
}

/* walls: the same velocity difference L_y gamma_dot(t) across the box, split -/+ */
double orc_wall_speed(const orc_params *p, int64_t t) {
  double s, u;
  le_protocol(p, t, &s, &u);
  return 0.5 * u;
}

/* ---------------- derived constants (Sec. 2) ---------------- */
int orc_resolve(const orc_params *p, int32_t np, const double *radius, orc_derived *d) {
  double amin = 0, amax = 0, msum = 0;
  for (int i = 0; i < np; ++i) {
    double a = radius[i];
    if (i == 0 || a < amin) amin = a;
    if (i == 0 || a > amax) amax = a;
    msum += p->rho_p * (4.0 / 3.0) * PI * a * a * a;
  }
  d->a_min = amin; d->a_max = amax;
  d->m0 = np > 0 ? msum / np : 0.0;
  /* dt = 0.6 tau_c with tau_c = sqrt(m0/kn) and dt = 1 gives kn = 0.36 m0 */
  d->kn = p->kn > 0 ? p->kn : 0.36 * d->m0;
  d->kt = p->kt_ratio * d->kn;
  d->eta_n = p->eta_n >= 0 ? p->eta_n : sqrt(d->m0 * d->kn);
  d->lub_delta = p->lub_delta >= 0 ? p->lub_delta : 0.01 * amin;
  d->debye_lambda = p->debye_lambda > 0 ? p->debye_lambda : 0.02 * amin;
  d->F0 = p->F0 >= 0 ? p->F0 : 2e-4 * d->kn;
  d->eta0 = p->rho0 * (p->tau - 0.5) / 3.0;
  return 0;
}

/* ---------------- pair interactions ---------------- */
static void cross(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Linear spring-dashpot normal force, Cundall-Strack tangential spring with Coulomb cap
 * (Sec. 2: F_nor = (kn delta_n + eta_n u_n) n, kt spring, |F_tan| <= mu |F_nor|), torque
 * eq. (11t).  n points from j to i; the contact point of i is R_i - a_i n.               */
int orc_contact(const orc_params *p, const orc_derived *d, double ai, double aj,
                const double dv[3], const double Ui[3], const double Uj[3],
                const double Wi[3], const double Wj[3], double dt, double xi[3],
                double Fi[3], double Ti[3], double Tj[3], double Fn_out[3]) {
  double r2 = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
  double r = sqrt(r2);
  double h = r - ai - aj;
  for (int c = 0; c < 3; ++c) { Fi[c] = 0; Ti[c] = 0; Tj[c] = 0; Fn_out[c] = 0; }
  if (!(h < 0.0)) { xi[0] = xi[1] = xi[2] = 0.0; return 0; }
  double n[3] = {dv[0] / r, dv[1] / r, dv[2] / r};
  double Uij[3] = {Ui[0] - Uj[0], Ui[1] - Uj[1], Ui[2] - Uj[2]};
  double vn = -dot(Uij, n);                   /* approach speed */
  double fnm = d->kn * (-h) + d->eta_n * vn;  /* signed normal magnitude, along n */
  double Fn[3] = {fnm * n[0], fnm * n[1], fnm * n[2]};
  /* relative velocity of the contact points */
  double aw[3] = {ai * Wi[0] + aj * Wj[0], ai * Wi[1] + aj * Wj[1], ai * Wi[2] + aj * Wj[2]};
  double awn[3];
  cross(aw, n, awn);
  double v[3] = {Uij[0] - awn[0], Uij[1] - awn[1], Uij[2] - awn[2]};
  double vdn = dot(v, n);
  double vt[3] = {v[0] - vdn * n[0], v[1] - vdn * n[1], v[2] - vdn * n[2]};
  /* rotate the spring into the current tangent plane, keeping its length */
  double xn = dot(xi, n);
  double xp[3] = {xi[0] - xn * n[0], xi[1] - xn * n[1], xi[2] - xn * n[2]};
  double mo = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
  double mp = sqrt(xp[0] * xp[0] + xp[1] * xp[1] + xp[2] * xp[2]);
  if (mp > 0.0) {
    double sc = mo / mp;
    xi[0] = xp[0] * sc; xi[1] = xp[1] * sc; xi[2] = xp[2] * sc;
  } else {
    xi[0] = xp[0]; xi[1] = xp[1]; xi[2] = xp[2];
  }
  xi[0] += vt[0] * dt; xi[1] += vt[1] * dt; xi[2] += vt[2] * dt;
  double Ft[3] = {-d->kt * xi[0], -d->kt * xi[1], -d->kt * xi[2]};
  double ftm = sqrt(Ft[0] * Ft[0] + Ft[1] * Ft[1] + Ft[2] * Ft[2]);
  double cap = p->mu * fabs(fnm);
  if (ftm > cap) {
    double sc = cap / ftm;
    Ft[0] *= sc; Ft[1] *= sc; Ft[2] *= sc;
    xi[0] = -Ft[0] / d->kt; xi[1] = -Ft[1] / d->kt; xi[2] = -Ft[2] / d->kt;
  }
  for (int c = 0; c < 3; ++c) { Fi[c] = Fn[c] + Ft[c]; Fn_out[c] = Fn[c]; }
  double li[3] = {-ai * n[0], -ai * n[1], -ai * n[2]};
  double lj[3] = {-aj * n[0], -aj * n[1], -aj * n[2]};
  cross(li, Ft, Ti);
  cross(lj, Ft, Tj);
  return 1;
}

/* eq. (13): F_r = F0 exp(-h/lambda) n, with the gap clamped at 0. */
void orc_dlvo(const orc_params *p, const orc_derived *d, double ai, double aj,
              const double dv[3], double Fi[3]) {
  double r2 = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
  double r = sqrt(r2);
  double h = r - ai - aj;
  Fi[0] = Fi[1] = Fi[2] = 0.0;
  if (!(h < p->pair_cutoff)) return;
  double hh = h > 0.0 ? h : 0.0;
  double f = d->F0 * exp(-hh / d->debye_lambda);
  Fi[0] = f * dv[0] / r; Fi[1] = f * dv[1] / r; Fi[2] = f * dv[2] / r;
}

/* Leading-order scalar resistance functions of App. A for the block of sphere "a" with
 * partner ratio b (b = partner radius / own radius); inv = 1/xi, lg = ln(1/xi) terms.    */
typedef struct { double XA, YA, YB, XG, YG, YC, YCp, YH, YHp; } lubfun;
static lubfun lub_block(double a, double b, double inv, double lg) {
  lubfun f;
  double b1 = 1.0 + b;
  f.XA = 6.0 * PI * a * (2.0 * b * b / (b1 * b1 * b1)) * inv;
  f.YA = 6.0 * PI * a * (4.0 * b * (2.0 + b + 2.0 * b * b) / (15.0 * b1 * b1 * b1)) * lg;
  f.YB = 4.0 * PI * a * a * (b * (4.0 + b) / (5.0 * b1 * b1)) * lg;
  f.XG = 4.0 * PI * a * a * (3.0 * b * b / (b1 * b1 * b1)) * inv;
  f.YG = 4.0 * PI * a * a * (b * (4.0 - b + 7.0 * b * b) / (10.0 * b1 * b1 * b1)) * lg;
  f.YC = 8.0 * PI * a * a * a * (2.0 * b / (5.0 * b1)) * lg;
  f.YCp = 8.0 * PI * a * a * a * (b * b / (10.0 * b1)) * lg;            /* C_ij */
  f.YH = 8.0 * PI * a * a * a * (b * (2.0 - b) / (10.0 * b1 * b1)) * lg;
  f.YHp = 8.0 * PI * a * a * a * (b * b * (1.0 + 7.0 * b) / (20.0 * b1 * b1)) * lg; /* H_ij */
  return f;
}

static void sym6(const double a[3], const double b[3], double w, double o[6]) {
  /* o += w (a b + b a) */
  o[0] += w * (2.0 * a[0] * b[0]);
  o[1] += w * (2.0 * a[1] * b[1]);
  o[2] += w * (2.0 * a[2] * b[2]);
  o[3] += w * (a[0] * b[1] + b[0] * a[1]);
  o[4] += w * (a[0] * b[2] + b[0] * a[2]);
  o[5] += w * (a[1] * b[2] + b[1] * a[2]);
}

/* Grand-resistance lubrication correction (App. A).  Readings: n points from j to i in
 * the force/torque rows; the stresslet rows carry the sign that makes a closing pair
 * compressive; beta of the ii block is a_j/a_i; every function is evaluated at
 * xi = 2(h+delta)/(a_i+a_j) and, with lub_subtract_hc, minus its value at h = h_c.      */
void orc_lubrication(const orc_params *p, const orc_derived *d, double ai, double aj,
                     const double dv[3], const double Ui[3], const double Uj[3],
                     const double Wi[3], const double Wj[3], double Fi[3], double Ti[3],
                     double Tj[3], double Si[6], double Sj[6]) {
  for (int c = 0; c < 3; ++c) { Fi[c] = 0; Ti[c] = 0; Tj[c] = 0; }
  for (int c = 0; c < 6; ++c) { Si[c] = 0; Sj[c] = 0; }
  double r2 = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
  double r = sqrt(r2);
  double h = r - ai - aj;
  if (!(h < p->lub_hc)) return;
  double n[3] = {dv[0] / r, dv[1] / r, dv[2] / r};
  double hh = h > 0.0 ? h : 0.0;
  double xg = 2.0 * (hh + d->lub_delta) / (ai + aj);
  double inv = 1.0 / xg, lg = log(1.0 / xg);
  if (p->lub_subtract_hc) {
    double xc = 2.0 * (p->lub_hc + d->lub_delta) / (ai + aj);
    inv = inv - 1.0 / xc;
    lg = lg - log(1.0 / xc);
  }
  lubfun fi = lub_block(ai, aj / ai, inv, lg);
  lubfun fj = lub_block(aj, ai / aj, inv, lg);
  double eta = d->eta0;
  double U[3] = {Ui[0] - Uj[0], Ui[1] - Uj[1], Ui[2] - Uj[2]};
  double un = dot(U, n);
  double Wixn[3], Wjxn[3], Uxn[3];
  cross(Wi, n, Wixn);
  cross(Wj, n, Wjxn);
  cross(U, n, Uxn);
  double wi_n = dot(Wi, n), wj_n = dot(Wj, n);
  for (int c = 0; c < 3; ++c) {
    double AU = fi.XA * un * n[c] + fi.YA * (U[c] - un * n[c]);
    /* F_i = -eta (A_ii U - B_ii W_i + B_jj W_j); B(n) W = YB (W x n), B_jj uses -n */
    Fi[c] = -eta * (AU - fi.YB * Wixn[c] - fj.YB * Wjxn[c]);
    double Wip = Wi[c] - wi_n * n[c], Wjp = Wj[c] - wj_n * n[c];
    /* T_i = -eta (B_ii U + C_ii W_i + C_ij W_j) */
    Ti[c] = -eta * (fi.YB * Uxn[c] + fi.YC * Wip + fi.YCp * Wjp);
    /* T_j = -eta (-B_jj U + C_ij W_i + C_jj W_j) */
    Tj[c] = -eta * (fj.YB * Uxn[c] + fi.YCp * Wip + fj.YC * Wjp);
  }
  /* stresslets: S = -eta (G U + H W + H' W'), G odd in its normal, H even. */
  double s1[6] = {0, 0, 0, 0, 0, 0}; /* (n n - I/3)(n.U) */
  double s2[6] = {0, 0, 0, 0, 0, 0}; /* n U + U n - 2 n n (n.U) */
  double hi[6] = {0, 0, 0, 0, 0, 0}; /* (W_i x n) n + n (W_i x n) */
  double hj[6] = {0, 0, 0, 0, 0, 0};
  sym6(n, n, 0.5 * un, s1);
  s1[0] -= un / 3.0; s1[1] -= un / 3.0; s1[2] -= un / 3.0;
  sym6(n, U, 1.0, s2);
  sym6(n, n, -un, s2);
  sym6(Wixn, n, 1.0, hi);
  sym6(Wjxn, n, 1.0, hj);
  for (int c = 0; c < 6; ++c) {
    /* G_ii evaluated with the normal from i to j (= -n) */
    double Gi = -(fi.XG * s1[c] + fi.YG * s2[c]);
    Si[c] = -eta * (Gi + fi.YH * hi[c] + fi.YHp * hj[c]);
    /* -G_jj with the normal from j to i (= n) */
    double Gj = -(fj.XG * s1[c] + fj.YG * s2[c]);
    Sj[c] = -eta * (Gj + fj.YHp * hi[c] + fj.YH * hj[c]);
  }
}

/* ---------------- simulation object ---------------- */
static void *xcalloc(size_t n, size_t sz) {
  void *q = calloc(n ? n : 1, sz);
  return q;
}

static void quat_step(double *Q, const double W[3], double dt) {
  /* q <- normalize(q + dt/2 (0, W) (x) q) */
  double qw = Q[0], qx = Q[1], qy = Q[2], qz = Q[3];
  double dw = -(W[0] * qx + W[1] * qy + W[2] * qz);
  double dx = W[0] * qw + (W[1] * qz - W[2] * qy);
  double dy = W[1] * qw + (W[2] * qx - W[0] * qz);
  double dz = W[2] * qw + (W[0] * qy - W[1] * qx);
  qw += 0.5 * dt * dw; qx += 0.5 * dt * dx; qy += 0.5 * dt * dy; qz += 0.5 * dt * dz;
  double nn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  Q[0] = qw / nn; Q[1] = qx / nn; Q[2] = qy / nn; Q[3] = qz / nn;
}

/* Candidate integer range around centre c with half-width r (superset of the sphere). */
static void cand_range(double c, double r, int L, int *lo, int *hi) {
  int a = (int)ceil(c - r - 1e-6), b = (int)floor(c + r + 1e-6);
  if (b - a + 1 >= L) { a = 0; b = L - 1; }
  *lo = a; *hi = b;
}

/* Mapped-sphere membership of a lattice point (x,y,z) (y may be -1 or ly) for particle p
 * at position Rp = R[3p..3p+2] under offset s: strict |d|^2 < a_map^2.                    */
static int inside(const orc_sim *S, const double *R, int p, double s, double x, double y, double z) {
  double d[3];
  orc_minimage(&S->p, s, x - R[3 * p], y - R[3 * p + 1], z - R[3 * p + 2], d, NULL);
  double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  return r2 < S->amap[p] * S->amap[p];
}

/* Visit every node of particle p's mapped sphere (all images), calling fn(node). */
typedef void (*node_fn)(orc_sim *S, int p, int64_t node, int x, int y, int z, void *ctx);
static void for_footprint(orc_sim *S, const double *R, int p, double s, node_fn fn, void *ctx) {
  const orc_params *P = &S->p;
  double r = S->amap[p];
  for (int k = -1; k <= 1; ++k) {
    double cy = R[3 * p + 1] + k * (double)P->ly;
    double cx = R[3 * p] + k * s;
    int ylo = (int)ceil(cy - r - 1e-6), yhi = (int)floor(cy + r + 1e-6);
    if (ylo < 0) ylo = 0;
    if (yhi > P->ly - 1) yhi = P->ly - 1;
    if (ylo > yhi) continue;
    int xlo, xhi, zlo, zhi;
    cand_range(cx, r, P->lx, &xlo, &xhi);
    cand_range(R[3 * p + 2], r, P->lz, &zlo, &zhi);
    for (int zz = zlo; zz <= zhi; ++zz)
      for (int yy = ylo; yy <= yhi; ++yy)
        for (int xu = xlo; xu <= xhi; ++xu) {
          int x = wrapi(xu, P->lx), z = wrapi(zz, P->lz);
          int32_t kk;
          double dd[3];
          orc_minimage(P, s, x - R[3 * p], yy - R[3 * p + 1], z - R[3 * p + 2], dd, &kk);
          if (kk != k) continue; /* reached through a different image box */
          if (!(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2] < S->amap[p] * S->amap[p])) continue;
          int64_t node = x + (int64_t)P->lx * (yy + (int64_t)P->ly * z);
          fn(S, p, node, x, yy, z, ctx);
        }
  }
}

static void claim_fn(orc_sim *S, int p, int64_t node, int x, int y, int z, void *ctx) {
  (void)x; (void)y; (void)z;
  int32_t *own = (int32_t *)ctx;
  if (own[node] == -2) return;
  if (own[node] >= 0 && own[node] != p) {
    S->flags |= 1;
    if (p < own[node]) own[node] = p;
    return;
  }
  own[node] = p;
}

static void build_map(orc_sim *S, int32_t *own, const double *R, double s) {
  const orc_params *P = &S->p;
  for (int64_t i = 0; i < S->nodes; ++i) own[i] = -1;
  if (P->wall_y)
    for (int z = 0; z < P->lz; ++z)
      for (int x = 0; x < P->lx; ++x) {
        own[x + (int64_t)P->lx * (0 + (int64_t)P->ly * z)] = -2;
        own[x + (int64_t)P->lx * ((P->ly - 1) + (int64_t)P->ly * z)] = -2;
      }
  for (int p = 0; p < S->np; ++p) for_footprint(S, R, p, s, claim_fn, own);
}

int orc_remap(orc_sim *S) {
  S->flags = 0;
  build_map(S, S->own, S->R, S->s_next);
  return 0;
}

orc_sim *orc_create(const orc_params *p, int32_t np, const double *pos, const double *vel,
                    const double *omega, const double *radius) {
  orc_sim *S = (orc_sim *)xcalloc(1, sizeof(orc_sim));
  S->p = *p;
  orc_resolve(p, np, radius, &S->d);
  S->nodes = (int64_t)p->lx * p->ly * p->lz;
  S->f = (double *)xcalloc((size_t)19 * S->nodes, sizeof(double));
  S->fn = (double *)xcalloc((size_t)19 * S->nodes, sizeof(double));
  S->own = (int32_t *)xcalloc((size_t)S->nodes, sizeof(int32_t));
  S->np = np;
  S->R = (double *)xcalloc(3 * (size_t)np, sizeof(double));
  S->U = (double *)xcalloc(3 * (size_t)np, sizeof(double));
  S->W = (double *)xcalloc(3 * (size_t)np, sizeof(double));
  S->Q = (double *)xcalloc(4 * (size_t)np, sizeof(double));
  S->a = (double *)xcalloc((size_t)np, sizeof(double));
  S->m = (double *)xcalloc((size_t)np, sizeof(double));
  S->I = (double *)xcalloc((size_t)np, sizeof(double));
  S->amap = (double *)xcalloc((size_t)np, sizeof(double));
  S->Fh = (double *)xcalloc(3 * (size_t)np, sizeof(double));
  S->Th = (double *)xcalloc(3 * (size_t)np, sizeof(double));
  S->Sh = (double *)xcalloc(9 * (size_t)np, sizeof(double));
  S->nlinks = (int32_t *)xcalloc((size_t)np, sizeof(int32_t));
  S->Frest = (double *)xcalloc(3 * (size_t)np, sizeof(double));
  S->Trest = (double *)xcalloc(3 * (size_t)np, sizeof(double));
  S->gown = (int32_t *)xcalloc(2 * (size_t)p->lx * p->lz, sizeof(int32_t));
  S->cst = (double *)xcalloc(3 * (size_t)(p->contact_bins > 0 ? p->contact_bins : 1), sizeof(double));
  S->wall = (int32_t *)xcalloc((size_t)(np > 0 ? np : 1), sizeof(int32_t));
  for (int i = 0; i < np; ++i) {
    for (int c = 0; c < 3; ++c) {
      S->R[3 * i + c] = pos[3 * i + c];
      S->U[3 * i + c] = vel ? vel[3 * i + c] : 0.0;
      S->W[3 * i + c] = omega ? omega[3 * i + c] : 0.0;
    }
    S->Q[4 * i] = 1.0;
    double a = radius[i];
    S->a[i] = a;
    S->m[i] = p->rho_p * (4.0 / 3.0) * PI * a * a * a;
    S->I[i] = 0.4 * S->m[i] * a * a;
    S->amap[i] = p->map_ratio * a;
  }
#ifdef _OPENMP
  S->nthreads = omp_get_max_threads();
#else
  S->nthreads = 1;
#endif
  /* initial fluid: equilibrium at rho0 and the affine profile of the shear at t = 0 */
  double s0, u0;
  orc_protocol(p, 0, &s0, &u0);
  S->s_next = s0;
  double gd = (p->boundary == 1 ? 2.0 * orc_wall_speed(p, 0) : u0) / (double)p->ly;
  for (int z = 0; z < p->lz; ++z)
    for (int y = 0; y < p->ly; ++y)
      for (int x = 0; x < p->lx; ++x) {
        int64_t node = x + (int64_t)p->lx * (y + (int64_t)p->ly * z);
        double ux = gd * ((double)y - 0.5 * (double)(p->ly - 1));
        double fe[19];
        orc_feq(p->rho0, ux, 0.0, 0.0, fe);
        for (int q = 0; q < 19; ++q) S->f[q * S->nodes + node] = fe[q];
      }
  build_map(S, S->own, S->R, S->s_next);
  return S;
}

void orc_destroy(orc_sim *S) {
  if (!S) return;
  free(S->f); free(S->fn); free(S->own); free(S->R); free(S->U); free(S->W); free(S->Q);
  free(S->a); free(S->m); free(S->I); free(S->amap); free(S->Fh); free(S->Th); free(S->Sh);
  free(S->nlinks); free(S->Frest); free(S->Trest); free(S->pi); free(S->pj); free(S->hi); free(S->hj); free(S->hxi);
  free(S->gown); free(S->cst); free(S->wall);
  free(S);
}

int orc_set_history(orc_sim *S, int32_t n, const int32_t *i, const int32_t *j, const double *xi) {
  free(S->hi); free(S->hj); free(S->hxi);
  S->nhist = n; S->hist_cap = n;
  S->hi = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
  S->hj = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
  S->hxi = (double *)xcalloc(3 * (size_t)n, sizeof(double));
  for (int k = 0; k < n; ++k) {
    S->hi[k] = i[k]; S->hj[k] = j[k];
    S->hxi[3 * k] = xi[3 * k]; S->hxi[3 * k + 1] = xi[3 * k + 1]; S->hxi[3 * k + 2] = xi[3 * k + 2];
  }
  return 0;
}

/* ---------------- ghost planes for the Lees-Edwards boundary ---------------- */
typedef struct {
  double *val;   /* [2][5][lz][lx] interpolated, Galilean-corrected populations */
} ghost_t;

/* Galilean-corrected post-collision value of direction q at node (x,yrow,z) as seen from the
 * image box: sgn=+1 for the box below (velocity shifted by -U_LE), -1 for the box above.  */
static double nhat(const orc_sim *S, int q, int x, int yrow, int z, double s, double ule, int sgn) {
  const orc_params *P = &S->p;
  int64_t node = x + (int64_t)P->lx * (yrow + (int64_t)P->ly * z);
  int o = S->own[node];
  if (o >= 0) {
    double d[3]; int32_t k;
    orc_minimage(P, s, x - S->R[3 * o], yrow - S->R[3 * o + 1], z - S->R[3 * o + 2], d, &k);
    const double *W = &S->W[3 * o];
    double ub[3] = {S->U[3 * o] + k * ule + (W[1] * d[2] - W[2] * d[1]),
                    S->U[3 * o + 1] + (W[2] * d[0] - W[0] * d[2]),
                    S->U[3 * o + 2] + (W[0] * d[1] - W[1] * d[0])};
    return feq1(q, P->rho0, ub[0] - sgn * ule, ub[1], ub[2]);
  }
  double rho = 0, jx = 0, jy = 0, jz = 0;
  for (int r = 0; r < 19; ++r) {
    double v = S->f[r * S->nodes + node];
    rho += v; jx += v * CX[r]; jy += v * CY[r]; jz += v * CZ[r];
  }
  double ux = jx / rho, uy = jy / rho, uz = jz / rho;
  double fq = S->f[q * S->nodes + node];
  return fq + (feq1(q, rho, ux - sgn * ule, uy, uz) - feq1(q, rho, ux, uy, uz));
}

static void build_ghosts(orc_sim *S, double s, double ule, ghost_t *G) {
  const orc_params *P = &S->p;
  int lx = P->lx, lz = P->lz;
  for (int i = 0; i < 2 * lx * lz; ++i) S->gown[i] = -1;
  /* owners: geometric test of the points (x,-1,z) and (x,ly,z) against particle images */
  for (int p = 0; p < S->np; ++p) {
    double r = S->amap[p];
    for (int g = 0; g < 2; ++g) {
      double gy = g == 0 ? -1.0 : (double)P->ly;
      for (int k = -1; k <= 1; ++k) {
        double cy = S->R[3 * p + 1] + k * (double)P->ly;
        if (!(fabs(gy - cy) < r + 1e-6)) continue;
        double cx = S->R[3 * p] + k * s;
        int xlo, xhi, zlo, zhi;
        cand_range(cx, r, lx, &xlo, &xhi);
        cand_range(S->R[3 * p + 2], r, lz, &zlo, &zhi);
        for (int zz = zlo; zz <= zhi; ++zz)
          for (int xu = xlo; xu <= xhi; ++xu) {
            int x = wrapi(xu, lx), z = wrapi(zz, lz);
            if (!inside(S, S->R, p, s, x, gy, z)) continue;
            int32_t *o = &S->gown[g * lx * lz + z * lx + x];
            if (*o >= 0 && *o != p) { S->flags |= 1; if (p < *o) *o = p; }
            else *o = p;
          }
      }
    }
  }
  /* values at fluid ghost points: linear interpolation along x of the shifted row */
  for (int g = 0; g < 2; ++g) {
    const int *qs = g == 0 ? UPQ : DNQ;
    int yrow = g == 0 ? P->ly - 1 : 0;
    int sgn = g == 0 ? 1 : -1;
    for (int z = 0; z < lz; ++z)
      for (int x = 0; x < lx; ++x) {
        double xs = (double)x + sgn * s;
        double x0f = floor(xs);
        double fr = xs - x0f;
        int i0 = wrapi((int)x0f, lx), i1 = wrapi((int)x0f + 1, lx);
        for (int m = 0; m < 5; ++m) {
          double v0 = nhat(S, qs[m], i0, yrow, z, s, ule, sgn);
          double v1 = nhat(S, qs[m], i1, yrow, z, s, ule, sgn);
          G->val[((g * 5 + m) * lz + z) * lx + x] = (1.0 - fr) * v0 + fr * v1;
        }
      }
  }
}

/* ---------------- one LB step of the fluid with particle links ---------------- */
/* per-particle link sums: F[3] T[3] S[9] count, rest-state force[3] and torque[3] */
#define ACC 22

static void fluid_step(orc_sim *S, double s, double ule, const ghost_t *G, double pineq[6],
                       double wflat[6]) {
  const orc_params *P = &S->p;
  const int lx = P->lx, ly = P->ly, lz = P->lz, np = S->np;
  const int64_t nodes = S->nodes;
  const double rho0 = P->rho0, tau = P->tau;
  int nt = S->nthreads;
  double *acc = (double *)xcalloc((size_t)nt * (np > 0 ? np : 1) * ACC, sizeof(double));
  double *pacc = (double *)xcalloc((size_t)nt * 6, sizeof(double));
  double *wacc = (double *)xcalloc((size_t)nt * 6, sizeof(double));
#pragma omp parallel num_threads(nt)
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    double *A = acc + (size_t)tid * (np > 0 ? np : 1) * ACC;
    double *pa = pacc + 6 * tid;
    double *pw = wacc + 6 * tid;
#pragma omp for schedule(static)
    for (int z = 0; z < lz; ++z)
      for (int y = 0; y < ly; ++y)
        for (int x = 0; x < lx; ++x) {
          int64_t X = x + (int64_t)lx * (y + (int64_t)ly * z);
          if (S->own[X] != -1) continue;
          double n[19];
          n[0] = S->f[X];
          for (int q = 1; q < 19; ++q) {
            int px = x - CX[q], py = y - CY[q], pz = z - CZ[q];
            if (P->boundary == 1 && (py < 0 || py >= ly)) {
              /* flat wall halfway between the edge row and its ghost, moving at -/+ U_w:
               * bounce-back with the wall velocity (eq. 7) */
              double uw = py < 0 ? -S->wspeed : S->wspeed;
              double fo = S->f[OPP(q) * nodes + X];
              n[q] = fo + 6.0 * WQ(q) * rho0 * uw * CX[q];
              /* momentum the wall receives, measured from the rest state rho0 */
              double mm = 2.0 * (fo - WQ(q) * rho0) + 6.0 * WQ(q) * rho0 * uw * CX[q];
              double *wf = pw + (py < 0 ? 0 : 3);
              wf[0] -= mm * CX[q]; wf[1] -= mm * CY[q]; wf[2] -= mm * CZ[q];
              continue;
            }
            int wx = wrapi(px, lx), wz = wrapi(pz, lz);
            int owner;
            double val = 0.0;
            if (py < 0 || py >= ly) {
              int g = py < 0 ? 0 : 1;
              owner = S->gown[g * lx * lz + wz * lx + wx];
              if (owner < 0) {
                int m = 0;
                const int *qs = g == 0 ? UPQ : DNQ;
                while (qs[m] != q) ++m;
                val = G->val[((g * 5 + m) * lz + wz) * lx + wx];
              }
            } else {
              int64_t Ps = wx + (int64_t)lx * (py + (int64_t)ly * wz);
              owner = S->own[Ps];
              if (owner == -1) val = S->f[q * nodes + Ps];
            }
            int co = OPP(q);
            double fo = S->f[co * nodes + X];
            if (owner == -1) {
              n[q] = val;
            } else if (owner == -2) {
              /* test-only static/moving wall */
              double uw = py <= 0 ? P->wall_u_bot : P->wall_u_top;
              double ubc = uw * CX[co];
              n[q] = fo - 6.0 * WQ(co) * rho0 * ubc;
            } else {
              /* eq. (7)-(8): bounce-back from the moving sphere surface halfway along the link */
              int p = owner;
              double d[3]; int32_t k;
              orc_minimage(P, s, px - S->R[3 * p], py - S->R[3 * p + 1], pz - S->R[3 * p + 2], d, &k);
              double lev[3] = {d[0] + 0.5 * CX[q], d[1] + 0.5 * CY[q], d[2] + 0.5 * CZ[q]};
              const double *Wp = &S->W[3 * p];
              double ub[3] = {S->U[3 * p] + k * ule + (Wp[1] * lev[2] - Wp[2] * lev[1]),
                              S->U[3 * p + 1] + (Wp[2] * lev[0] - Wp[0] * lev[2]),
                              S->U[3 * p + 2] + (Wp[0] * lev[1] - Wp[1] * lev[0])};
              double ubc = ub[0] * CX[co] + ub[1] * CY[co] + ub[2] * CZ[co];
              double corr = 6.0 * WQ(co) * rho0 * ubc;
              n[q] = fo - corr;
              /* eq. (6) (one factor 2): momentum exchanged across the link, measured from
               * the uniform rest state rho0 (whose part 2 w rho0 c is kept apart) */
              double fm = 2.0 * fo - corr;
              double fr = 2.0 * WQ(co) * rho0;
              double fc = fm - fr;
              double fl[3] = {fc * CX[co], fc * CY[co], fc * CZ[co]};
              double rl[3] = {fr * CX[co], fr * CY[co], fr * CZ[co]};
              double *a = A + ACC * (size_t)p;
              a[0] += fl[0]; a[1] += fl[1]; a[2] += fl[2];
              a[3] += lev[1] * fl[2] - lev[2] * fl[1];
              a[4] += lev[2] * fl[0] - lev[0] * fl[2];
              a[5] += lev[0] * fl[1] - lev[1] * fl[0];
              for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) a[6 + 3 * r + c] += lev[r] * fl[c];
              a[15] += 1.0;
              a[16] += rl[0]; a[17] += rl[1]; a[18] += rl[2];
              a[19] += lev[1] * rl[2] - lev[2] * rl[1];
              a[20] += lev[2] * rl[0] - lev[0] * rl[2];
              a[21] += lev[0] * rl[1] - lev[1] * rl[0];
            }
          }
          /* eq. (4) moments */
          double rho = 0, jx = 0, jy = 0, jz = 0;
          for (int q = 0; q < 19; ++q) {
            rho += n[q]; jx += n[q] * CX[q]; jy += n[q] * CY[q]; jz += n[q] * CZ[q];
          }
          double ux = jx / rho, uy = jy / rho, uz = jz / rho;
          double fe[19], ne[19];
          orc_feq(rho, ux, uy, uz, fe);
          for (int q = 0; q < 19; ++q) ne[q] = n[q] - fe[q];
          double Pn[3][3] = {{0}};  /* non-equilibrium momentum flux Pi^neq */
          for (int q = 0; q < 19; ++q) {
            const int c[3] = {CX[q], CY[q], CZ[q]};
            for (int a = 0; a < 3; ++a)
              for (int b = 0; b < 3; ++b) Pn[a][b] += ne[q] * c[a] * c[b];
          }
          pa[0] += Pn[0][0]; pa[1] += Pn[1][1]; pa[2] += Pn[2][2];
          pa[3] += Pn[0][1]; pa[4] += Pn[0][2]; pa[5] += Pn[1][2];
          /* eq. (5).  BGK: n* = n^eq + (1 - 1/tau) n^neq.  Linearised multi-eigenvalue form
           * (Ladd): with Q(M)_q = w_q (M : (c_q c_q - cs^2 I)) / (2 cs^4) the stress part of
           * a non-equilibrium distribution, the traceless part of Pi^neq is multiplied by
           * 1 + lambda, its trace by 1 + lambda_v, and the remainder n^neq - Q(Pi^neq) (the
           * ghost modes) by 1 + lambda_g; mass and momentum are unchanged.               */
          double post[19];
          if (P->collision == 1) {
            const double lam = -1.0 / tau, lamv = -1.0 / P->tau_bulk, lamg = -1.0 / P->tau_ghost;
            const double cs2 = 1.0 / 3.0;
            double tr = Pn[0][0] + Pn[1][1] + Pn[2][2];
            double Ps[3][3];
            for (int a = 0; a < 3; ++a)
              for (int b = 0; b < 3; ++b) {
                double dl = a == b ? 1.0 : 0.0;
                Ps[a][b] = (1.0 + lam) * (Pn[a][b] - dl * tr / 3.0) + (1.0 + lamv) * dl * tr / 3.0;
              }
            for (int q = 0; q < 19; ++q) {
              const int c[3] = {CX[q], CY[q], CZ[q]};
              double qs = 0.0, qn = 0.0;
              for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                  double h = c[a] * c[b] - (a == b ? cs2 : 0.0);
                  qs += Ps[a][b] * h;
                  qn += Pn[a][b] * h;
                }
              qs *= WQ(q) / (2.0 * cs2 * cs2);
              qn *= WQ(q) / (2.0 * cs2 * cs2);
              post[q] = fe[q] + qs + (1.0 + lamg) * (ne[q] - qn);
            }
          } else {
            for (int q = 0; q < 19; ++q) post[q] = n[q] - ne[q] / tau;
          }
          for (int q = 0; q < 19; ++q) {
            double v = post[q];
            if (P->gx != 0.0 || P->gy != 0.0 || P->gz != 0.0)
              v += 3.0 * WQ(q) * (CX[q] * P->gx + CY[q] * P->gy + CZ[q] * P->gz);
            S->fn[q * nodes + X] = v;
          }
        }
  }
  /* fixed-order reduction of the per-thread partials */
  for (int p = 0; p < np; ++p) {
    double t[ACC] = {0};
    for (int th = 0; th < nt; ++th)
      for (int c = 0; c < ACC; ++c) t[c] += acc[((size_t)th * np + p) * ACC + c];
    for (int c = 0; c < 3; ++c) { S->Fh[3 * p + c] = t[c]; S->Th[3 * p + c] = t[3 + c]; }
    for (int c = 0; c < 9; ++c) S->Sh[9 * p + c] = t[6 + c];
    S->nlinks[p] = (int32_t)t[15];
    for (int c = 0; c < 3; ++c) { S->Frest[3 * p + c] = t[16 + c]; S->Trest[3 * p + c] = t[19 + c]; }
  }
  for (int c = 0; c < 6; ++c) {
    pineq[c] = 0;
    wflat[c] = 0;
    for (int th = 0; th < nt; ++th) { pineq[c] += pacc[6 * th + c]; wflat[c] += wacc[6 * th + c]; }
  }
  free(acc);
  free(pacc);
  free(wacc);
  double *t = S->f; S->f = S->fn; S->fn = t;
}

/* ---------------- pairs ---------------- */
static void build_pairs(orc_sim *S, double s) {
  const int np = S->np;
  const double hl = S->p.pair_cutoff;
  int32_t *cnt = (int32_t *)xcalloc((size_t)np + 1, sizeof(int32_t));
  int32_t **lst = (int32_t **)xcalloc((size_t)np, sizeof(int32_t *));
  int ovl = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : ovl) if (np > 64)
  for (int i = 0; i < np; ++i) {
    int cap = 16, c = 0;
    int32_t *L = (int32_t *)malloc(cap * sizeof(int32_t));
    for (int j = i + 1; j < np; ++j) {
      double d[3];
      orc_minimage(&S->p, s, S->R[3 * i] - S->R[3 * j], S->R[3 * i + 1] - S->R[3 * j + 1],
                   S->R[3 * i + 2] - S->R[3 * j + 2], d, NULL);
      double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      double rc = S->a[i] + S->a[j] + hl;
      if (r2 < rc * rc) {
        if (c == cap) { cap *= 2; L = (int32_t *)realloc(L, cap * sizeof(int32_t)); }
        L[c++] = j;
        double rm = S->amap[i] + S->amap[j];
        if (r2 < rm * rm) ovl = 1;
      }
    }
    lst[i] = L; cnt[i] = c;
  }
  if (ovl) S->flags |= 1;
  int64_t tot = 0;
  for (int i = 0; i < np; ++i) tot += cnt[i];
  if (tot > S->pairs_cap) {
    free(S->pi); free(S->pj);
    S->pairs_cap = (int32_t)tot;
    S->pi = (int32_t *)xcalloc((size_t)tot, sizeof(int32_t));
    S->pj = (int32_t *)xcalloc((size_t)tot, sizeof(int32_t));
  }
  int64_t k = 0;
  for (int i = 0; i < np; ++i) {
    for (int c = 0; c < cnt[i]; ++c) { S->pi[k] = i; S->pj[k] = lst[i][c]; ++k; }
    free(lst[i]);
  }
  S->npairs = (int32_t)tot;
  free(lst);
  free(cnt);
}

static int find_hist(const orc_sim *S, int i, int j) {
  int lo = 0, hi = S->nhist - 1;
  while (lo <= hi) {
    int mid = (lo + hi) / 2;
    int a = S->hi[mid], b = S->hj[mid];
    if (a == i && b == j) return mid;
    if (a < i || (a == i && b < j)) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

/* ---------------- map update: covered and uncovered nodes ---------------- */
typedef struct {
  const int32_t *own_other; /* covers: map before the move; uncovers: map after the move */
  const double *R, *U, *W;  /* particle state after the move */
  double s, ule;            /* offset and sliding velocity after the move */
  double *dp;               /* [7 np]: momentum, angular momentum, fluid mass */
} remap_ctx;

/* A node that was fluid and is now inside particle p: its fluid is absorbed. */
static void cover_fn(orc_sim *S, int p, int64_t node, int x, int y, int z, void *vctx) {
  remap_ctx *c = (remap_ctx *)vctx;
  if (c->own_other[node] != -1) return;
  double rho = 0, j[3] = {0, 0, 0};
  for (int q = 0; q < 19; ++q) {
    double v = S->f[q * S->nodes + node];
    rho += v; j[0] += v * CX[q]; j[1] += v * CY[q]; j[2] += v * CZ[q];
  }
  double d[3]; int32_t k;
  orc_minimage(&S->p, c->s, x - c->R[3 * p], y - c->R[3 * p + 1], z - c->R[3 * p + 2], d, &k);
  j[0] -= rho * k * c->ule; /* momentum seen from the particle's own image frame */
  double *a = c->dp + 7 * (size_t)p;
  a[0] += j[0]; a[1] += j[1]; a[2] += j[2];
  a[3] += d[1] * j[2] - d[2] * j[1];
  a[4] += d[2] * j[0] - d[0] * j[2];
  a[5] += d[0] * j[1] - d[1] * j[0];
  a[6] += rho;
}

/* A node inside particle p before the move and fluid after it: refilled with the
 * equilibrium at rho0 and the surface velocity; the particle pays that momentum.     */
static void uncover_fn(orc_sim *S, int p, int64_t node, int x, int y, int z, void *vctx) {
  remap_ctx *c = (remap_ctx *)vctx;
  if (c->own_other[node] != -1) return;
  double d[3]; int32_t k;
  orc_minimage(&S->p, c->s, x - c->R[3 * p], y - c->R[3 * p + 1], z - c->R[3 * p + 2], d, &k);
  const double *W = &c->W[3 * p];
  double ub[3] = {c->U[3 * p] + (W[1] * d[2] - W[2] * d[1]),
                  c->U[3 * p + 1] + (W[2] * d[0] - W[0] * d[2]),
                  c->U[3 * p + 2] + (W[0] * d[1] - W[1] * d[0])};
  double fe[19];
  orc_feq(S->p.rho0, ub[0] + k * c->ule, ub[1], ub[2], fe);
  for (int q = 0; q < 19; ++q) S->f[q * S->nodes + node] = fe[q];
  double r0 = S->p.rho0;
  double j[3] = {r0 * ub[0], r0 * ub[1], r0 * ub[2]};
  double *a = c->dp + 7 * (size_t)p;
  a[0] -= j[0]; a[1] -= j[1]; a[2] -= j[2];
  a[3] -= d[1] * j[2] - d[2] * j[1];
  a[4] -= d[2] * j[0] - d[0] * j[2];
  a[5] -= d[0] * j[1] - d[1] * j[0];
  a[6] -= r0;
}

static int finite3(const double *v) { return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]); }

/* ---------------- the full step ---------------- */
/* Squeeze coefficient of the pair (the X^A term of the force on i in orc_lubrication). */
double orc_lub_squeeze(const orc_params *p, const orc_derived *d, double ai, double aj,
                       const double dv[3]) {
  double r = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  double h = r - ai - aj;
  if (!(h < p->lub_hc)) return 0.0;
  double hh = h > 0.0 ? h : 0.0;
  double xg = 2.0 * (hh + d->lub_delta) / (ai + aj);
  double inv = 1.0 / xg, lg = log(1.0 / xg);
  if (p->lub_subtract_hc) {
    double xc = 2.0 * (p->lub_hc + d->lub_delta) / (ai + aj);
    inv = inv - 1.0 / xc;
    lg = lg - log(1.0 / xc);
  }
  lubfun fi = lub_block(ai, aj / ai, inv, lg);
  return d->eta0 * fi.XA;
}

/* x = A^-1 r for a symmetric positive definite 3x3 A (Cramer's rule). */
static void solve3(const double A[3][3], const double r[3], double x[3]) {
  double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
  double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
  double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
  double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
  double inv[3][3] = {
      {c00, A[0][2] * A[2][1] - A[0][1] * A[2][2], A[0][1] * A[1][2] - A[0][2] * A[1][1]},
      {c01, A[0][0] * A[2][2] - A[0][2] * A[2][0], A[0][2] * A[1][0] - A[0][0] * A[1][2]},
      {c02, A[0][1] * A[2][0] - A[0][0] * A[2][1], A[0][0] * A[1][1] - A[0][1] * A[1][0]}};
  for (int a = 0; a < 3; ++a) x[a] = (inv[a][0] * r[0] + inv[a][1] * r[1] + inv[a][2] * r[2]) / det;
}

void orc_implicit_solve(int32_t n, const double *m, const int32_t *fixed, const double *b,
                        int32_t npairs, const int32_t *pi, const int32_t *pj, const double *zeta,
                        const double *nv, const double *sh, double dt, int32_t sweeps, double *U) {
  double *A = (double *)xcalloc(9 * (size_t)(n > 0 ? n : 1), sizeof(double));
  double *r = (double *)xcalloc(3 * (size_t)(n > 0 ? n : 1), sizeof(double));
  double *Un = (double *)xcalloc(3 * (size_t)(n > 0 ? n : 1), sizeof(double));
  for (int s = 0; s < sweeps; ++s) {
    for (int i = 0; i < n; ++i) {
      for (int c = 0; c < 9; ++c) A[9 * i + c] = (c % 4 == 0) ? m[i] : 0.0;
      for (int c = 0; c < 3; ++c) r[3 * i + c] = b[3 * i + c];
    }
    for (int k = 0; k < npairs; ++k) {
      int i = pi[k], j = pj[k];
      const double *nk = &nv[3 * k], *sk = &sh[3 * k];
      double w = dt * zeta[k];
      /* row i: the partner's image moves at U_j + s_k; row j: the partner at U_i - s_k */
      double uj = nk[0] * (U[3 * j] + sk[0]) + nk[1] * (U[3 * j + 1] + sk[1]) + nk[2] * (U[3 * j + 2] + sk[2]);
      double ui = nk[0] * (U[3 * i] - sk[0]) + nk[1] * (U[3 * i + 1] - sk[1]) + nk[2] * (U[3 * i + 2] - sk[2]);
      for (int a = 0; a < 3; ++a) {
        for (int c = 0; c < 3; ++c) {
          A[9 * i + 3 * a + c] += w * nk[a] * nk[c];
          A[9 * j + 3 * a + c] += w * nk[a] * nk[c];
        }
        r[3 * i + a] += w * nk[a] * uj;
        r[3 * j + a] += w * nk[a] * ui;
      }
    }
    for (int i = 0; i < n; ++i) {
      if (fixed && fixed[i]) { for (int c = 0; c < 3; ++c) Un[3 * i + c] = U[3 * i + c]; continue; }
      double Ai[3][3] = {{A[9 * i], A[9 * i + 1], A[9 * i + 2]},
                         {A[9 * i + 3], A[9 * i + 4], A[9 * i + 5]},
                         {A[9 * i + 6], A[9 * i + 7], A[9 * i + 8]}};
      solve3(Ai, &r[3 * i], &Un[3 * i]);
    }
    memcpy(U, Un, 3 * sizeof(double) * (size_t)n);
  }
  free(A); free(r); free(Un);
}

/* ---------------- contact statistics (Sec. 4.2, eqs. 19-23) ----------------
 * A contact is a pair whose surfaces overlap at the last DEM substep of a step; dv = R_i - R_j
 * (minimum image), Fn and Fc the normal and the total contact force on i at that substep.
 * Orientation: theta = atan(r_y / r_x) of the in-plane part of dv, in [0, pi) (the contact
 * seen from either sphere is one orientation); a contact with no in-plane part counts at 0.
 * F_nor: the normal force, positive when it pushes the spheres apart.  F_tan: the component
 * along t_theta = (-sin theta, cos theta) of the tangential force on the sphere at the tail
 * of n_theta, positive when it turns that sphere counterclockwise.  Seen from the other
 * sphere n_theta, t_theta and the force all reverse, so both values are the same.          */
static void contact_sample(orc_sim *S, const double dv[3], const double Fn[3], const double Fc[3]) {
  const int nb = S->p.contact_bins;
  double r = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  double rxy = sqrt(dv[0] * dv[0] + dv[1] * dv[1]);
  double nx = 1.0, ny = 0.0;
  if (rxy > 0.0) { nx = dv[0] / rxy; ny = dv[1] / rxy; }
  double fnor = (Fn[0] * dv[0] + Fn[1] * dv[1] + Fn[2] * dv[2]) / r;
  double ft[3] = {Fc[0] - Fn[0], Fc[1] - Fn[1], Fc[2] - Fn[2]};
  /* n_theta = dv / |dv| points from j to i, so the sphere at its tail is j, which feels -ft */
  double ftan = -(ft[0] * (-ny) + ft[1] * nx);
  double ox = nx, oy = ny;
  if (oy < 0.0 || (oy == 0.0 && ox < 0.0)) { ox = -ox; oy = -oy; }
  double th = atan2(oy, ox);
  int b = (int)(th * (double)nb / PI);
  if (b < 0) b = 0;
  if (b > nb - 1) b = nb - 1;
  S->cst[3 * b] += 1.0;
  S->cst[3 * b + 1] += fnor;
  S->cst[3 * b + 2] += ftan;
  S->ctot[0] += 1.0;
  S->ctot[1] += fnor;
  /* integrand of eqs. 26-27: [F_nor n - F_tan t] (x) n with n = (nx, ny), t = (-ny, nx) */
  double vx = fnor * nx - ftan * (-ny), vy = fnor * ny - ftan * nx;
  S->ctot[2] += vx * nx; S->ctot[3] += vx * ny; S->ctot[4] += vy * nx; S->ctot[5] += vy * ny;
}

static void one_step(orc_sim *S) {
  orc_params *P = &S->p;
  const int np = S->np;
  const size_t npa = np > 0 ? (size_t)np : 1;
  double s, ule, s1, ule1;
  orc_protocol(P, S->step, &s, &ule);
  orc_protocol(P, S->step + 1, &s1, &ule1);
  S->s = s; S->ule = ule;
  const double V = (double)P->lx * P->ly * P->lz;
  double *R0 = (double *)xcalloc(3 * npa, sizeof(double));
  memcpy(R0, S->R, 3 * sizeof(double) * (size_t)np);

  /* neighbour list from the positions at the start of the step, history carried over */
  build_pairs(S, s);
  size_t npp = S->npairs > 0 ? (size_t)S->npairs : 1;
  double *pxi = (double *)xcalloc(3 * npp, sizeof(double));
  int32_t *pon = (int32_t *)xcalloc(npp, sizeof(int32_t));
  for (int k = 0; k < S->npairs; ++k) {
    int h = find_hist(S, S->pi[k], S->pj[k]);
    if (h >= 0) {
      pxi[3 * k] = S->hxi[3 * h]; pxi[3 * k + 1] = S->hxi[3 * h + 1]; pxi[3 * k + 2] = S->hxi[3 * h + 2];
      pon[k] = 1;
    }
  }

  /* fluid: Lees-Edwards ghosts (or moving walls), then stream + bounce-back + collide with
   * link forces */
  const int walls = P->boundary == 1;
  S->wspeed = walls ? orc_wall_speed(P, S->step) : 0.0;
  const double wsp1 = walls ? orc_wall_speed(P, S->step + 1) : 0.0;
  ghost_t G;
  G.val = (double *)xcalloc((size_t)2 * 5 * P->lx * P->lz, sizeof(double));
  if (walls) {
    for (int i = 0; i < 2 * P->lx * P->lz; ++i) S->gown[i] = -1;
  } else {
    build_ghosts(S, s, ule, &G);
  }
  double pineq[6], wflat[6];
  fluid_step(S, s, ule, &G, pineq, wflat);
  free(G.val);
  double wf[2][3] = {{wflat[0], wflat[1], wflat[2]}, {wflat[3], wflat[4], wflat[5]}};
  if (walls)
    for (int i = 0; i < np; ++i)
      if (S->wall[i] > 0)
        for (int c = 0; c < 3; ++c) wf[S->wall[i] - 1][c] += S->Fh[3 * i + c];

  /* DEM substeps: eq. (1) with the hydrodynamic force and torque frozen over the step */
  double *Fp = (double *)xcalloc(3 * npa, sizeof(double));
  double *Tp = (double *)xcalloc(3 * npa, sizeof(double));
  double sc[6] = {0}, sr[6] = {0}, sl[6] = {0};
  const int ns = P->n_sub;
  const double dts = 1.0 / (double)ns;
  /* implicit squeeze terms: per pair zeta, n, image shift; per sphere the squeeze force at
   * the old velocities (for the explicit first guess) */
  const int imp = P->lub_implicit > 0;
  double *zk = (double *)xcalloc(npp, sizeof(double));
  double *nk = (double *)xcalloc(3 * npp, sizeof(double));
  double *sk = (double *)xcalloc(3 * npp, sizeof(double));
  double *Fq = (double *)xcalloc(3 * npa, sizeof(double));
  double *bq = (double *)xcalloc(3 * npa, sizeof(double));
  double *Uq = (double *)xcalloc(3 * npa, sizeof(double));
  int32_t *fixq = (int32_t *)xcalloc(npa, sizeof(int32_t));
  for (int sub = 0; sub < ns; ++sub) {
    memset(Fp, 0, 3 * sizeof(double) * npa);
    memset(Tp, 0, 3 * sizeof(double) * npa);
    memset(Fq, 0, 3 * sizeof(double) * npa);
    for (int k = 0; k < S->npairs; ++k) {
      int i = S->pi[k], j = S->pj[k];
      double d[3]; int32_t kk;
      orc_minimage(P, s, S->R[3 * i] - S->R[3 * j], S->R[3 * i + 1] - S->R[3 * j + 1],
                   S->R[3 * i + 2] - S->R[3 * j + 2], d, &kk);
      double Uj[3] = {S->U[3 * j] + kk * ule, S->U[3 * j + 1], S->U[3 * j + 2]};
      const double *Ui = &S->U[3 * i], *Wi = &S->W[3 * i], *Wj = &S->W[3 * j];
      double Fc[3], Tci[3], Tcj[3], Fn[3], Fr[3], Fl[3], Tli[3], Tlj[3], Si[6], Sj[6];
      pon[k] = orc_contact(P, &S->d, S->a[i], S->a[j], d, Ui, Uj, Wi, Wj, dts, &pxi[3 * k],
                           Fc, Tci, Tcj, Fn);
      if (P->contact_bins > 0 && sub == ns - 1 && pon[k]) contact_sample(S, d, Fn, Fc);
      orc_dlvo(P, &S->d, S->a[i], S->a[j], d, Fr);
      orc_lubrication(P, &S->d, S->a[i], S->a[j], d, Ui, Uj, Wi, Wj, Fl, Tli, Tlj, Si, Sj);
      double Fs[3] = {0.0, 0.0, 0.0};
      if (imp) {
        /* the squeeze part of Fl, -zeta n (n . (U_i - U_j)), leaves the explicit sum */
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double nn[3] = {d[0] / r, d[1] / r, d[2] / r};
        double z = orc_lub_squeeze(P, &S->d, S->a[i], S->a[j], d);
        double un = nn[0] * (Ui[0] - Uj[0]) + nn[1] * (Ui[1] - Uj[1]) + nn[2] * (Ui[2] - Uj[2]);
        zk[k] = z;
        for (int c = 0; c < 3; ++c) { nk[3 * k + c] = nn[c]; Fs[c] = -z * un * nn[c]; }
        sk[3 * k] = kk * ule; sk[3 * k + 1] = 0.0; sk[3 * k + 2] = 0.0;
        for (int c = 0; c < 3; ++c) { Fq[3 * i + c] += Fs[c]; Fq[3 * j + c] -= Fs[c]; }
      }
      for (int c = 0; c < 3; ++c) {
        double F = Fc[c] + Fr[c] + (Fl[c] - Fs[c]);
        Fp[3 * i + c] += F; Fp[3 * j + c] -= F;
        Tp[3 * i + c] += Tci[c] + Tli[c];
        Tp[3 * j + c] += Tcj[c] + Tlj[c];
      }
      /* eqs. (12), (14) counted once per pair: -(1/V) sym(r_ij (x) F_ij); stresslets + */
      sym6(d, Fc, -0.5 / V, sc);
      sym6(d, Fr, -0.5 / V, sr);
      for (int c = 0; c < 6; ++c) sl[c] += (Si[c] + Sj[c]) / V;
    }
    if (imp) {
      /* m U' + dt sum zeta n n . (U' - U'_j) = m U + dt (F^h + explicit pair forces),
       * started from the explicit update */
      for (int i = 0; i < np; ++i) {
        fixq[i] = walls && S->wall[i] > 0;
        for (int c = 0; c < 3; ++c) {
          bq[3 * i + c] = S->m[i] * S->U[3 * i + c] + dts * (S->Fh[3 * i + c] + Fp[3 * i + c]);
          Uq[3 * i + c] = fixq[i] ? S->U[3 * i + c]
                                  : S->U[3 * i + c] + dts * (S->Fh[3 * i + c] + Fp[3 * i + c] + Fq[3 * i + c]) / S->m[i];
        }
      }
      orc_implicit_solve(np, S->m, fixq, bq, S->npairs, S->pi, S->pj, zk, nk, sk, dts, P->lub_implicit, Uq);
    }
    for (int i = 0; i < np; ++i) {
      double *U = &S->U[3 * i], *W = &S->W[3 * i], *R = &S->R[3 * i];
      if (walls && S->wall[i] > 0) {
        /* a wall sphere moves with its wall; the pair forces on it load the wall */
        for (int c = 0; c < 3; ++c) wf[S->wall[i] - 1][c] += Fp[3 * i + c] / (double)ns;
        U[0] = S->wall[i] == 2 ? S->wspeed : -S->wspeed;
        U[1] = 0.0; U[2] = 0.0; W[0] = 0.0; W[1] = 0.0; W[2] = 0.0;
        R[0] += dts * U[0];
        continue;
      }
      for (int c = 0; c < 3; ++c) {
        U[c] = imp ? Uq[3 * i + c] : U[c] + dts * (S->Fh[3 * i + c] + Fp[3 * i + c]) / S->m[i];
        W[c] += dts * (S->Th[3 * i + c] + Tp[3 * i + c]) / S->I[i];
      }
      if (P->quasi2d) { U[2] = 0.0; W[0] = 0.0; W[1] = 0.0; }
      for (int c = 0; c < 3; ++c) R[c] += dts * U[c];
      quat_step(&S->Q[4 * i], W, dts);
    }
  }
  free(Fp);
  free(Tp);
  free(zk); free(nk); free(sk); free(Fq); free(bq); free(Uq); free(fixq);
  /* surviving contacts become the new history (already in (i,j) order) */
  int nh = 0;
  for (int k = 0; k < S->npairs; ++k) nh += pon[k] ? 1 : 0;
  free(S->hi); free(S->hj); free(S->hxi);
  S->hi = (int32_t *)xcalloc((size_t)nh, sizeof(int32_t));
  S->hj = (int32_t *)xcalloc((size_t)nh, sizeof(int32_t));
  S->hxi = (double *)xcalloc(3 * (size_t)nh, sizeof(double));
  S->nhist = nh; S->hist_cap = nh;
  nh = 0;
  for (int k = 0; k < S->npairs; ++k)
    if (pon[k]) {
      S->hi[nh] = S->pi[k]; S->hj[nh] = S->pj[k];
      S->hxi[3 * nh] = pxi[3 * k]; S->hxi[3 * nh + 1] = pxi[3 * k + 1]; S->hxi[3 * nh + 2] = pxi[3 * k + 2];
      ++nh;
    }
  free(pxi);
  free(pon);

  if (walls) {
    /* the walls' velocity for the next step; a free sphere leaving the gap is a failure */
    for (int i = 0; i < np; ++i) {
      if (S->wall[i] > 0) S->U[3 * i] = S->wall[i] == 2 ? wsp1 : -wsp1;
      else if (!(S->R[3 * i + 1] >= 0.0 && S->R[3 * i + 1] < (double)P->ly)) S->flags |= 2;
    }
    for (int g = 0; g < 2; ++g)
      for (int c = 0; c < 3; ++c) S->wforce[g][c] += wf[g][c];
    S->wcount += 1;
  }
  /* Lees-Edwards wrap of the particles with the offset of the next step */
  for (int i = 0; i < np; ++i) {
    double *R = &S->R[3 * i], *U = &S->U[3 * i];
    if (walls) {
    } else if (R[1] >= P->ly) { R[1] -= P->ly; R[0] -= s1; U[0] -= ule1; }
    else if (R[1] < 0.0) { R[1] += P->ly; R[0] += s1; U[0] += ule1; }
    for (int it = 0; it < 4 && R[0] >= P->lx; ++it) R[0] -= P->lx;
    for (int it = 0; it < 4 && R[0] < 0.0; ++it) R[0] += P->lx;
    for (int it = 0; it < 4 && R[2] >= P->lz; ++it) R[2] -= P->lz;
    for (int it = 0; it < 4 && R[2] < 0.0; ++it) R[2] += P->lz;
  }

  /* map update: new footprints absorb fluid nodes, old footprints release nodes */
  if (np > 0) {
    int32_t *own_new = (int32_t *)xcalloc((size_t)S->nodes, sizeof(int32_t));
    build_map(S, own_new, S->R, s1);
    double *dp = (double *)xcalloc(7 * npa, sizeof(double));
    remap_ctx cc = {S->own, S->R, S->U, S->W, s1, ule1, dp};
    for (int p = 0; p < np; ++p) for_footprint(S, S->R, p, s1, cover_fn, &cc);
    remap_ctx uc = {own_new, S->R, S->U, S->W, s1, ule1, dp};
    for (int p = 0; p < np; ++p) for_footprint(S, R0, p, s, uncover_fn, &uc);
    for (int p = 0; p < np; ++p) {
      const double *a = dp + 7 * (size_t)p;
      if (walls && S->wall[p] > 0) {  /* prescribed motion: the impulses load the wall */
        for (int c = 0; c < 3; ++c) S->wforce[S->wall[p] - 1][c] += a[c];
        S->ledger += a[6];
        continue;
      }
      for (int c = 0; c < 3; ++c) {
        S->U[3 * p + c] += a[c] / S->m[p];
        S->W[3 * p + c] += a[3 + c] / S->I[p];
      }
      if (P->quasi2d) { S->U[3 * p + 2] = 0.0; S->W[3 * p] = 0.0; S->W[3 * p + 1] = 0.0; }
      S->ledger += a[6];
    }
    free(S->own);
    S->own = own_new;
    free(dp);
  }
  free(R0);
  for (int i = 0; i < np; ++i)
    if (!finite3(&S->R[3 * i]) || !finite3(&S->U[3 * i]) || !finite3(&S->W[3 * i])) S->flags |= 2;

  /* stress of this step, eq. (15) with the fluid, particle and lubrication parts */
  double sig[5][6];
  /* fluid stress: the mean of the non-equilibrium momentum flux before and after collision,
   * -(1 + lambda/2) for the traceless part and -(1 + lambda_v/2) for the trace */
  double cf = -(1.0 - 0.5 / P->tau) / V;
  for (int c = 0; c < 6; ++c) sig[0][c] = cf * pineq[c];
  if (P->collision == 1) {
    double cb = -(1.0 - 0.5 / P->tau_bulk) / V;
    double t3 = (pineq[0] + pineq[1] + pineq[2]) / 3.0;
    for (int c = 0; c < 3; ++c) sig[0][c] = cf * (pineq[c] - t3) + cb * t3;
  }
  double sh[6] = {0, 0, 0, 0, 0, 0};
  for (int p = 0; p < np; ++p) {
    const double *m = &S->Sh[9 * p];
    sh[0] += m[0]; sh[1] += m[4]; sh[2] += m[8];
    sh[3] += 0.5 * (m[1] + m[3]); sh[4] += 0.5 * (m[2] + m[6]); sh[5] += 0.5 * (m[5] + m[7]);
  }
  for (int c = 0; c < 6; ++c) {
    sig[1][c] = sh[c] / V;
    sig[2][c] = sl[c] / ns;
    sig[3][c] = sc[c] / ns;
    sig[4][c] = sr[c] / ns;
  }
  for (int k = 0; k < 5; ++k)
    for (int c = 0; c < 6; ++c) { S->sig_last[k][c] = sig[k][c]; S->sig_sum[k][c] += sig[k][c]; }
  S->sig_count += 1;
  if (P->contact_bins > 0) {
    for (int c = 0; c < 6; ++c) S->csig[c] += sig[0][c] + sig[1][c] + sig[2][c] + sig[3][c] + sig[4][c];
    S->csamples += 1;
  }
  /* G', G'' (eqs. 17-18, rectangle rule over the observation periods) */
  {
    double wc, ws;
    if (orc_gg_weight(P, S->step, &wc, &ws)) {
      double sxy = sig[0][3] + sig[1][3] + sig[2][3] + sig[3][3] + sig[4][3];
      S->gp_cos += sxy * wc;
      S->gp_sin += sxy * ws;
      S->gp_count += 1;
    }
  }
  S->step += 1;
  S->s_next = s1;
}

int orc_step(orc_sim *S, int64_t nsteps) {
  for (int64_t t = 0; t < nsteps; ++t) {
    one_step(S);
    if (S->flags) return -4;
  }
  return 0;
}

void orc_stress(orc_sim *S, double out[5][6], double gg[2]) {
  double n = S->sig_count > 0 ? (double)S->sig_count : 1.0;
  for (int k = 0; k < 5; ++k)
    for (int c = 0; c < 6; ++c) { out[k][c] = S->sig_sum[k][c] / n; S->sig_sum[k][c] = 0.0; }
  S->sig_count = 0;
  orc_gg_moduli(&S->p, S->gp_cos, S->gp_sin, S->gp_count, gg);
}

/* Eqs. (17)-(18) as a rectangle rule over whole observation periods of P steps: the
 * integral (omega/pi) int_0^{2 pi/omega} dt f(t) over N periods becomes (2/(N P)) sum_t f(t).
 * Step t enters with the phase omega (t - t_I) + Theta of eq. (16) (t_I = ncyc_I periods:
 * the observation cycles restart the strain at the amplitude g0_F). */
int orc_gg_weight(const orc_params *p, int64_t t, double *wc, double *ws) {
  *wc = 0.0; *ws = 0.0;
  if (p->shear_kind != 2) return 0;
  int64_t tI = (int64_t)p->ncyc_I * p->period, tF = tI + (int64_t)p->ncyc_F * p->period;
  if (t < tI || t >= tF) return 0;
  double om = 2.0 * PI / (double)p->period;
  double ph = om * (double)(t - tI) + p->theta;
  *wc = cos(ph);
  *ws = sin(ph);
  return 1;
}

/* G' = -(2 / (n g0_F)) sum sigma_xy cos(phase), G'' = (2 / (n g0_F)) sum sigma_xy sin(phase)
 * over the n observation steps summed so far (eqs. 17, 18); zero before the first. */
void orc_gg_moduli(const orc_params *p, double sum_cos, double sum_sin, int64_t n, double gg[2]) {
  if (n > 0 && p->g0_F != 0.0) {
    double c = 2.0 / ((double)n * p->g0_F);
    gg[0] = -c * sum_cos;
    gg[1] = c * sum_sin;
  } else {
    gg[0] = 0.0; gg[1] = 0.0;
  }
}

/* G', G'' of a given shear-stress history: sxy[k] is the stress of step t0 + k. */
void orc_gg_series(const orc_params *p, int64_t t0, int64_t n, const double *sxy, double gg[2]) {
  double sc = 0.0, ss = 0.0;
  int64_t cnt = 0;
  for (int64_t k = 0; k < n; ++k) {
    double wc, ws;
    if (orc_gg_weight(p, t0 + k, &wc, &ws)) { sc += sxy[k] * wc; ss += sxy[k] * ws; cnt += 1; }
  }
  orc_gg_moduli(p, sc, ss, cnt, gg);
}

void orc_quat_step(double q[4], const double W[3], double dt) { quat_step(q, W, dt); }

int orc_set_walls(orc_sim *S, const int32_t *member) {
  const orc_params *P = &S->p;
  double h = 0.5 * P->pair_cutoff;
  for (int i = 0; i < S->np; ++i) {
    int m = member[i];
    if (m < 0 || m > 2) return -1;
    double y = S->R[3 * i + 1], a = S->a[i];
    if (m == 1 && !(y > a + h)) return -1;
    if (m == 2 && !(y < (double)P->ly - a - h)) return -1;
  }
  double u = orc_wall_speed(P, S->step);
  for (int i = 0; i < S->np; ++i) {
    S->wall[i] = member[i];
    if (member[i] > 0) {
      S->U[3 * i] = member[i] == 2 ? u : -u;
      S->U[3 * i + 1] = 0.0; S->U[3 * i + 2] = 0.0;
      S->W[3 * i] = 0.0; S->W[3 * i + 1] = 0.0; S->W[3 * i + 2] = 0.0;
    }
  }
  return 0;
}

void orc_wall_force(orc_sim *S, double out[6]) {
  double n = S->wcount > 0 ? (double)S->wcount : 1.0;
  for (int g = 0; g < 2; ++g)
    for (int c = 0; c < 3; ++c) { out[3 * g + c] = S->wforce[g][c] / n; S->wforce[g][c] = 0.0; }
  S->wcount = 0;
}

/* Eigenvalues of a symmetric 3x3 matrix by cyclic Jacobi rotations, sorted descending. */
void orc_sym3_eigen(const double a6[6], double ev[3]) {
  double A[3][3] = {{a6[0], a6[3], a6[4]}, {a6[3], a6[1], a6[5]}, {a6[4], a6[5], a6[2]}};
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    if (off == 0.0) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (A[p][q] == 0.0) continue;
        /* rotation in the (p, q) plane that zeroes A[p][q] */
        double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < 3; ++k) {  /* columns p, q */
          double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - sn * akq;
          A[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {  /* rows p, q */
          double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - sn * aqk;
          A[q][k] = sn * apk + c * aqk;
        }
      }
  }
  ev[0] = A[0][0]; ev[1] = A[1][1]; ev[2] = A[2][2];
  for (int i = 0; i < 3; ++i)
    for (int k = i + 1; k < 3; ++k)
      if (ev[k] > ev[i]) { double x = ev[i]; ev[i] = ev[k]; ev[k] = x; }
}

/* Distributions of eqs. 19-23 per bin, the stress of eq. 27 (3D) or eq. 26 (monolayer) and
 * the anisotropy Delta lambda / P of the mean total stress, over the steps since the last call.
 * The integral of eqs. 26-27 is taken over the contacts themselves, i.e. <F_nor> times the
 * integral of [zeta_N n - zeta_T t] n equals the mean of [F_nor n - F_tan t] n over contacts.
 * Prefactor: the one for which the formula equals the contact virial of eq. 12 when every
 * contact is between spheres of radius a at distance 2a: 3 phi3 Z / (4 pi a^2) in 3D (App. C)
 * and phi Z / (pi a) per unit area in a monolayer (eq. 26), divided by lz to give a stress per
 * unit volume like eq. 15.  a is the mean radius, Z = 2 contacts / spheres.              */
int orc_contact_stats(orc_sim *S, int32_t nbins, double *hist, double summary[12]) {
  const orc_params *P = &S->p;
  if (nbins <= 0 || nbins != P->contact_bins) return -1;
  const double dth = PI / (double)nbins;
  const double nc = S->ctot[0];
  const double fmean = nc > 0.0 ? S->ctot[1] / nc : 0.0;  /* <F_nor> */
  for (int b = 0; b < nbins; ++b) {
    double c = S->cst[3 * b];
    double rho = nc > 0.0 ? c / (nc * dth) : 0.0;                 /* eq. 23 normalisation */
    double fnor = c > 0.0 ? S->cst[3 * b + 1] / c : 0.0;         /* F_nor(theta)          */
    double ftan = c > 0.0 ? S->cst[3 * b + 2] / c : 0.0;         /* F_tan(theta)          */
    double xn = fmean != 0.0 ? fnor / fmean : 0.0;               /* eq. 21                */
    double xt = fmean != 0.0 ? ftan / fmean : 0.0;               /* eq. 22                */
    hist[b] = rho;
    hist[nbins + b] = xn;
    hist[2 * nbins + b] = xt;
    hist[3 * nbins + b] = rho * xn;                               /* eq. 19                */
    hist[4 * nbins + b] = rho * xt;                               /* eq. 20                */
  }
  const double samples = (double)S->csamples;
  const int np = S->np;
  double Z = (np > 0 && samples > 0.0) ? 2.0 * nc / ((double)np * samples) : 0.0;
  double asum = 0.0, a2 = 0.0, a3 = 0.0;
  for (int i = 0; i < np; ++i) {
    asum += S->a[i];
    a2 += PI * S->a[i] * S->a[i];
    a3 += (4.0 / 3.0) * PI * S->a[i] * S->a[i] * S->a[i];
  }
  double am = np > 0 ? asum / (double)np : 0.0;
  double frac, C;
  if (P->quasi2d) {
    frac = a2 / ((double)P->lx * (double)P->ly);
    C = am > 0.0 ? frac * Z / (PI * am) / (double)P->lz : 0.0;
  } else {
    frac = a3 / ((double)P->lx * (double)P->ly * (double)P->lz);
    C = am > 0.0 ? 3.0 * frac * Z / (4.0 * PI * am * am) : 0.0;
  }
  double sh[4];
  for (int k = 0; k < 4; ++k) sh[k] = nc > 0.0 ? C * (S->ctot[2 + k] / nc) : 0.0;
  /* stress anisotropy of the mean total stress: Delta lambda = largest - smallest eigenvalue,
   * P = minus the mean eigenvalue (3D); the x-y block in a monolayer */
  double M[6];
  for (int c = 0; c < 6; ++c) M[c] = samples > 0.0 ? S->csig[c] / samples : 0.0;
  double dl, pr;
  if (P->quasi2d) {
    double mid = 0.5 * (M[0] + M[1]);
    double rad = sqrt(0.25 * (M[0] - M[1]) * (M[0] - M[1]) + M[3] * M[3]);
    dl = 2.0 * rad;
    pr = -mid;
  } else {
    double ev[3];
    orc_sym3_eigen(M, ev);
    dl = ev[0] - ev[2];
    pr = -(ev[0] + ev[1] + ev[2]) / 3.0;
  }
  summary[0] = samples;
  summary[1] = samples > 0.0 ? nc / samples : 0.0;
  summary[2] = Z;
  summary[3] = fmean;
  summary[4] = sh[0]; summary[5] = sh[1]; summary[6] = sh[2]; summary[7] = sh[3];
  summary[8] = dl;
  summary[9] = pr;
  summary[10] = pr != 0.0 ? dl / pr : 0.0;
  summary[11] = frac;
  memset(S->cst, 0, 3 * sizeof(double) * (size_t)nbins);
  memset(S->ctot, 0, sizeof S->ctot);
  memset(S->csig, 0, sizeof S->csig);
  S->csamples = 0;
  return 0;
}
