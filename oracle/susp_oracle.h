/*
 * susp_oracle.h -- plain FP64 CPU reference of one lattice-Boltzmann + DEM time step
 * for a sheared suspension of frictional spheres (Pradipto & Hayakawa, arXiv:1904.02929).
 *
 * TEST INFRASTRUCTURE ONLY.  This oracle exists to check the GPU library.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or helper with the GPU path.
 *
 * Units are lattice units (dx = dt = 1).  Nodes sit at integer coordinates (x,y,z),
 * 0 <= x < lx etc., linear index x + lx*(y + ly*z).  Populations are stored
 * direction-major: f[q*nodes + node].  The stored population state is the
 * post-collision distribution n* of every fluid node (values at solid nodes are ignored).
 */
#ifndef SUSP_ORACLE_H
#define SUSP_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t lx, ly, lz;
  double tau, rho0;            /* BGK relaxation time, reference density              */
  double map_ratio;            /* mapped radius / contact radius (0.95)               */
  double rho_p;                /* particle density                                    */
  double kn;                   /* normal spring; <= 0 -> 0.36 m0 (dt = 0.6 sqrt(m0/kn)) */
  double kt_ratio, mu;         /* kt = kt_ratio kn ; Coulomb coefficient              */
  double eta_n;                /* normal dashpot; < 0 -> sqrt(m0 kn)                  */
  double lub_delta;            /* roughness length; < 0 -> 0.01 a_min                 */
  double lub_hc;               /* lubrication acts for h < lub_hc                     */
  int32_t lub_subtract_hc;     /* 1: each resistance function minus its value at h_c   */
  double F0;                   /* DLVO amplitude; < 0 -> 2e-4 kn                      */
  double debye_lambda;         /* DLVO decay length; < 0 -> 0.02 a_min                */
  double pair_cutoff;          /* neighbour-list gap cutoff h_list                    */
  int32_t n_sub;               /* DEM substeps per LB step                            */
  int32_t quasi2d;             /* 1: U_z = 0, Omega_x = Omega_y = 0                   */
  int32_t shear_kind;          /* 0 none, 1 simple, 2 oscillatory                     */
  double gamma_dot;            /* simple shear rate                                   */
  double g0_I, g0_F;           /* oscillatory amplitudes (initial, observation)       */
  int32_t period;              /* steps per oscillation period                        */
  double theta;                /* initial phase                                       */
  int32_t ncyc_I, ncyc_F;      /* initial and observation cycles                      */
  /* test-only geometry used by the oracle's own pins (never by the GPU path) */
  int32_t wall_y;              /* 1: rows y=0 and y=ly-1 are static/moving walls      */
  double wall_u_bot, wall_u_top;
  double gx, gy, gz;           /* uniform body force per node                         */
  int32_t contact_bins;        /* > 0: contact statistics (Sec. 4.2) in this many angular
                                  bins over [0, pi), sampled once per step              */
  int32_t collision;           /* 0: BGK (one eigenvalue -1/tau); 1: linearised operator
                                  with separate eigenvalues -1/tau (shear stress),
                                  -1/tau_bulk (trace of the stress), -1/tau_ghost (the
                                  nine non-hydrodynamic modes)                          */
  double tau_bulk, tau_ghost;
  int32_t lub_implicit;        /* 0: every pair force explicit in each substep; K > 0: the
                                  normal squeeze term of the lubrication force taken at the
                                  new velocities, solved by K Jacobi sweeps              */
  int32_t boundary;            /* 0: Lees-Edwards in y; 1: walls (Sec. 3): flat walls at
                                  y = -1/2 and ly - 1/2 moving at -/+ U_w(t) in x, carrying
                                  layers of wall spheres that move with them              */
} orc_params;

/* Fully resolved constants after defaults are applied. */
typedef struct {
  double m0, kn, kt, eta_n, lub_delta, F0, debye_lambda, eta0, a_min, a_max;
} orc_derived;

typedef struct {
  orc_params p;
  orc_derived d;
  int64_t nodes;
  double *f;          /* [19*nodes] post-collision populations (state)                */
  double *fn;         /* [19*nodes] scratch for the next state                        */
  int32_t *own;       /* [nodes] owner particle id, -1 fluid, -2 wall                  */
  int32_t np;
  double *R, *U, *W, *Q, *a; /* [3np] [3np] [3np] [4np] [np] */
  double *m, *I, *amap;      /* [np] */
  /* per-step hydrodynamic results */
  double *Fh, *Th, *Sh;      /* [3np] [3np] [9np] (Sh row-major lever (x) force)       */
  int32_t *nlinks;           /* [np] boundary links per particle in the last step      */
  double *Frest, *Trest;     /* [3np] rest-state part 2 w rho0 c of the link momentum,
                                excluded from Fh, Th, Sh (see fluid_step)              */
  /* neighbour list (step start): pairs i<j, sorted by (i,j) */
  int32_t npairs, pairs_cap;
  int32_t *pi, *pj;
  /* tangential spring history: pairs in contact, sorted by (i,j) */
  int32_t nhist, hist_cap;
  int32_t *hi, *hj;
  double *hxi;               /* [3*nhist] */
  /* ghost planes (last step): owner for y=-1 and y=ly, [2][lz][lx] */
  int32_t *gown;
  /* shear protocol */
  int64_t step;
  double s, ule;             /* LE offset and velocity used by the last step         */
  double s_next;             /* LE offset the current particle/map state refers to   */
  /* stress: per-step components and accumulated sums */
  double sig_last[5][6];     /* fluid, hydro, lubrication, contact, dlvo (xx yy zz xy xz yz) */
  double sig_sum[5][6];
  int64_t sig_count;
  double gp_cos, gp_sin; int64_t gp_count;
  double ledger;             /* fluid mass removed by covering minus mass restored    */
  int32_t flags;             /* 1 mapped-sphere overlap, 2 non-finite particle state  */
  int32_t nthreads;
  /* contact statistics since the last orc_contact_stats call */
  double *cst;               /* [contact_bins][3] contacts, sum F_nor, sum F_tan per bin */
  double ctot[6];            /* contacts, sum F_nor, sum of [F_nor n - F_tan t] (x) n
                                (xx, xy, yx, yy) over all contacts                     */
  double csig[6];            /* sum over sampled steps of the total stress (eq. 15)    */
  int64_t csamples;          /* sampled steps                                          */
  /* walls (boundary 1): membership of each sphere, 0 free, 1 bottom wall, 2 top wall;
   * force of the suspension on each wall summed over the steps since the last read-out */
  int32_t *wall;
  double wforce[2][3];
  int64_t wcount;
  double wspeed;             /* wall speed U_w of the current step                     */
} orc_sim;

/* D3Q19 lattice as used by the oracle (index q: velocity, weight, opposite). */
void orc_lattice(int32_t *cx, int32_t *cy, int32_t *cz, double *w, int32_t *opp);

int orc_resolve(const orc_params *p, int32_t np, const double *radius, orc_derived *d);
orc_sim *orc_create(const orc_params *p, int32_t np, const double *pos, const double *vel,
                    const double *omega, const double *radius);
void orc_destroy(orc_sim *s);
/* Advance nsteps LB steps. Returns 0, or -4 if the step raised an instability flag. */
int orc_step(orc_sim *s, int64_t nsteps);
/* Rebuild the owner map from the current particles and offset (no cover/uncover). */
int orc_remap(orc_sim *s);
/* Replace the tangential history. */
int orc_set_history(orc_sim *s, int32_t n, const int32_t *i, const int32_t *j, const double *xi);
/* Averages since the previous call; gg = {G', G''} over completed observation steps. */
void orc_stress(orc_sim *s, double out[5][6], double gg[2]);
/* Contact statistics (Sec. 4.2, eqs. 19-23, 26-27; App. C) over the steps since the previous
 * call, then reset.  hist[5][nbins] = rho, xi_N, xi_T, zeta_N, zeta_T at the bin centres
 * (nbins must equal contact_bins); summary[12] = samples, contacts per sample, Z, <F_nor>,
 * sigma_hat xx, xy, yx, yy, Delta lambda, P, Delta lambda / P, volume (area) fraction.
 * Returns -1 if nbins does not match, else 0.                                            */
int orc_contact_stats(orc_sim *s, int32_t nbins, double *hist, double summary[12]);
/* Walls (boundary 1): mark spheres as members of the bottom (1) or top (2) wall; their
 * velocity becomes the wall's.  Each member must keep a gap of pair_cutoff / 2 to its own
 * box face (centre y > a + cutoff / 2 for the bottom, < ly - a - cutoff / 2 for the top) so
 * that the two walls never meet through the periodic image.  Returns -1 if violated.     */
int orc_set_walls(orc_sim *s, const int32_t *member);
/* Wall speed U_w(t) = L_y gamma_dot(t) / 2 of the protocol (the top wall moves at +U_w). */
double orc_wall_speed(const orc_params *p, int64_t t);
/* Mean force per step of the suspension on the bottom and top walls (flat wall plus its
 * spheres: hydrodynamic force and the substep-mean pair forces) since the last call, then
 * reset: out = {bottom x y z, top x y z}.  The flat-wall part is measured from the rest
 * state rho0 (like the link sums).                                                        */
void orc_wall_force(orc_sim *s, double out[6]);
/* Normal squeeze coefficient zeta = eta0 X^A of the lubrication force on i (App. A), so that
 * its squeeze part is -zeta n (n . (U_i - U_j)); 0 beyond lub_hc.                         */
double orc_lub_squeeze(const orc_params *p, const orc_derived *d, double ai, double aj,
                       const double dvec[3]);
/* Velocities of one substep with the squeeze terms implicit: m_i U_i + dt sum_k zeta_k n_k
 * n_k . (U_i - U_j - s_k) = b_i for every free sphere i (pair k = (i, j), s_k the velocity
 * shift of j's image, the force on j opposite); fixed spheres keep U.  U holds the starting
 * guess and receives the result of `sweeps` Jacobi sweeps (3x3 solves per sphere).        */
void orc_implicit_solve(int32_t n, const double *m, const int32_t *fixed, const double *b,
                        int32_t npairs, const int32_t *pi, const int32_t *pj, const double *zeta,
                        const double *nvec, const double *shift, double dt, int32_t sweeps,
                        double *U);
/* G', G'' quadrature of eqs. (17)-(18) (rectangle rule over whole observation periods):
 * orc_gg_weight gives cos and sin of the phase of step t and returns 1 if step t lies in the
 * observation cycles (else 0); orc_gg_moduli turns the sums of sigma_xy times those weights
 * over n observation steps into gg = {G', G''}; orc_gg_series does both for a stress
 * history sxy[n] whose first entry is the stress of step t0.                              */
int orc_gg_weight(const orc_params *p, int64_t t, double *wc, double *ws);
void orc_gg_moduli(const orc_params *p, double sum_cos, double sum_sin, int64_t n, double gg[2]);
void orc_gg_series(const orc_params *p, int64_t t0, int64_t n, const double *sxy, double gg[2]);
/* One orientation update of a DEM substep: q <- normalize(q + dt/2 (0, W) (x) q), W the
 * angular velocity in the space frame (the update the particle step applies).             */
void orc_quat_step(double q[4], const double W[3], double dt);
/* Eigenvalues of a symmetric 3x3 matrix (xx yy zz xy xz yz), descending (Jacobi). */
void orc_sym3_eigen(const double a[6], double ev[3]);
/* LE protocol at step t: offset s (wrapped to [0,lx)) and sliding velocity. */
void orc_protocol(const orc_params *p, int64_t t, double *s, double *ule);

/* Building blocks exposed for the pins. */
void orc_feq(double rho, double ux, double uy, double uz, double out[19]);
void orc_minimage(const orc_params *p, double s, double dx, double dy, double dz,
                  double out[3], int32_t *k);
/* Lubrication on the pair (i,j); dvec = R_i - R_j (minimum image). Outputs the force on i,
 * the torques on i and j and the stresslets of i and j (xx yy zz xy xz yz).               */
void orc_lubrication(const orc_params *p, const orc_derived *d, double ai, double aj,
                     const double dvec[3], const double Ui[3], const double Uj[3],
                     const double Wi[3], const double Wj[3], double Fi[3], double Ti[3],
                     double Tj[3], double Si[6], double Sj[6]);
/* Contact (normal spring-dashpot, Cundall-Strack tangential spring with Coulomb cap).
 * xi is the spring history (in/out). Returns 1 if in contact (history kept), 0 if not.   */
int orc_contact(const orc_params *p, const orc_derived *d, double ai, double aj,
                const double dvec[3], const double Ui[3], const double Uj[3],
                const double Wi[3], const double Wj[3], double dt, double xi[3],
                double Fi[3], double Ti[3], double Tj[3], double Fn_out[3]);
/* DLVO double-layer repulsion on i. */
void orc_dlvo(const orc_params *p, const orc_derived *d, double ai, double aj,
              const double dvec[3], double Fi[3]);

#ifdef __cplusplus
}
#endif
#endif
