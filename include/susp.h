/*
 * susp.h -- C ABI of the MI355X lattice-Boltzmann + DEM library for sheared, frictional,
 * non-Brownian suspensions (Pradipto & Hayakawa, arXiv:1904.02929).
 *
 * One call of susp_step advances the coupled system by whole lattice-Boltzmann steps:
 *   - D3Q19 collide-and-stream (App. A, eqs. 3-5; collision single-time BGK, or the
 *     linearised operator with separate shear, bulk and ghost eigenvalues)
 *     with a Lees-Edwards sliding boundary in y (interpolated, Galilean-corrected ghost
 *     rows; periodic in x and z),
 *   - moving-sphere bounce-back on links cut by the mapped spheres (App. A, eqs. 7-8),
 *     with the exchanged momentum (eq. 6) summed into force, torque and stresslet per
 *     particle (eqs. 9-10),
 *   - cell-list neighbour search and pair forces: linear spring-dashpot normal contact,
 *     Cundall-Strack tangential spring with Coulomb cap (Sec. 2, eqs. 11, 11t), DLVO
 *     repulsion (eq. 13) and the leading-order lubrication correction (App. A),
 *   - the particle equations of motion (eq. 1) with DEM substeps,
 *   - the mapped-sphere node update (nodes covered and released as spheres move),
 *   - the stress of eq. (15) split into fluid, particle-surface, lubrication, contact and
 *     DLVO parts, and the G', G'' quadratures of eqs. (17)-(18).
 *
 * Units: lattice units, dx = dt = 1.  Node (x,y,z) has linear index x + lx*(y + ly*z).
 * Directions q = 0..18: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 = (+1,+1,0), (-1,-1,0),
 * (+1,-1,0), (-1,+1,0), (+1,0,+1), (-1,0,-1), (+1,0,-1), (-1,0,+1), (0,+1,+1),
 * (0,-1,-1), (0,+1,-1), (0,-1,+1); the opposite of odd q is q+1.
 *
 * Conventions common to every call:
 *   - Return value: a susp_status; 0 on success.  No exception or abort crosses the ABI.
 *     susp_last_error() gives a human-readable text for the calling thread's last error.
 *   - Host pointers are owned by the caller and only read or written during the call.
 *   - Device state is owned by the simulation object, carved out of one device block that
 *     the library allocates at susp_create, or out of a caller-provided workspace of at least
 *     susp_footprint_bytes() bytes (which then stays owned by the caller and must outlive the
 *     simulation).
 *   - All device work is enqueued on the HIP stream given at creation (NULL: the null
 *     stream).  susp_step is asynchronous except for the instability check at its end; the
 *     getters, setters and susp_stress synchronise the stream.
 */
#ifndef SUSP_H
#define SUSP_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct susp_sim susp_sim;

typedef enum {
  SUSP_OK = 0,
  SUSP_EINVAL = -1,     /* a parameter or argument is out of range                      */
  SUSP_ENOMEM = -2,     /* device allocation failed or workspace too small             */
  SUSP_EDEVICE = -3,    /* a HIP call failed                                            */
  SUSP_EUNSTABLE = -4,  /* mapped spheres overlap, non-finite particle state, a particle
                           exceeded the neighbour capacity, a node touches more than six
                           spheres, a sphere moved more than one node in one step, a
                           non-finite fluid density or velocity, or the fluid mass plus the
                           ledger of covered nodes drifted by more than 1e-2 of the box's
                           mass (spheres touching node to node leak ~2e-4 per 1000 steps) */
  SUSP_ESTATE = -5      /* a state buffer does not match the simulation                */
} susp_status;

typedef enum {
  SUSP_FP64 = 0,        /* populations stored and collided in FP64                      */
  SUSP_FP32 = 1,        /* deviations n_q - w_q rho0 stored in FP32, FP32 collision     */
  SUSP_FP16STORE = 2    /* deviations stored as FP16 of (n_q - w_q rho0)/w_q * 2^k,
                           FP32 collision                                               */
} susp_precision;

/* Problem statement (Sec. 2, Sec. 4.1, App. A).  A value below zero for kn, eta_n,
 * lub_delta, F0 or debye_lambda selects the paper's default:
 *   kn = 0.36 m0 (dt = 0.6 sqrt(m0/kn) with dt = 1), eta_n = sqrt(m0 kn),
 *   lub_delta = 0.01 a_min, F0 = 2e-4 kn, debye_lambda = 0.02 a_min,
 * with m0 the mean particle mass and a_min the smallest contact radius.                   */
typedef struct {
  int32_t lx, ly, lz;        /* lattice size; all >= 8, ly >= 3 (2 a_max + pair_cutoff)  */
  int32_t precision;         /* susp_precision                                           */
  double tau, rho0;          /* BGK relaxation time (> 0.5), reference density          */
  int32_t n;                 /* number of spheres (0 allowed)                            */
  const double *pos;         /* [n][3] centres, inside [0,lx) x [0,ly) x [0,lz)          */
  const double *vel;         /* [n][3] or NULL (zero)                                    */
  const double *omega;       /* [n][3] or NULL (zero)                                    */
  const double *radius;      /* [n] contact radii                                        */
  double map_ratio;          /* mapped radius / contact radius (paper: 0.95)             */
  double rho_p;              /* particle density                                         */
  double kn, kt_ratio, mu, eta_n;
  double lub_delta, lub_hc;  /* roughness length; lubrication acts for gaps below lub_hc */
  int32_t lub_subtract_hc;   /* 1: each resistance function minus its value at lub_hc   */
  double F0, debye_lambda;
  double pair_cutoff;        /* neighbour-list gap cutoff; DLVO acts below it            */
  int32_t n_sub;             /* DEM substeps per lattice step (>= 1)                     */
  int32_t quasi2d;           /* 1: monolayer, U_z = Omega_x = Omega_y = 0 (Sec. 4.1)     */
  int32_t shear_kind;        /* 0 none, 1 simple (gamma_dot), 2 oscillatory (eq. 16)     */
  double gamma_dot;
  double g0_I, g0_F;         /* strain amplitude of the initial and observation cycles  */
  int32_t period;            /* steps per oscillation period (omega = 2 pi / period)     */
  double theta;              /* initial phase Theta                                      */
  int32_t ncyc_I, ncyc_F;    /* initial and observation cycles                           */
  int32_t fp16_exp;          /* k of the FP16 storage scale 2^k (SUSP_FP16STORE only)    */
  int32_t brick_y, brick_z;  /* lattice-kernel brick of 64 x brick_y x brick_z nodes;
                                0 = chosen from the lattice size (brick_y a multiple of 4) */
  int32_t contact_bins;      /* 0: off; 1..360: contact statistics (susp_contact_stats)
                                sampled every step in this many orientation bins          */
  int32_t collision;         /* eq. (5): 0 single-time BGK (eigenvalue -1/tau); 1 the
                                linearised operator with eigenvalue -1/tau for the traceless
                                stress, -1/tau_bulk for its trace and -1/tau_ghost for the
                                nine non-hydrodynamic modes (mass and momentum conserved) */
  double tau_bulk, tau_ghost;  /* > 1/2 each (collision 1)                               */
  int32_t lub_implicit;      /* 0: every pair force explicit in the DEM substeps.  K in
                                1..64: the normal squeeze part -zeta n (n . (U_i - U_j)) of
                                each pair's lubrication force (zeta = eta0 X^A, App. A) is
                                taken at the substep's new velocities, solved by K Jacobi
                                sweeps from the explicit update; spins, the other forces and
                                the stresslets stay explicit.  With walls, the wall force
                                then omits the squeeze part on wall spheres.               */
  int32_t boundary;          /* 0: Lees-Edwards sliding boundary in y.  1: walls (Sec. 3):
                                flat walls halfway outside rows 0 and ly-1, moving in x at
                                -U_w and +U_w, U_w = ly gamma_dot(t) / 2 of the protocol,
                                with the spheres marked in `wall` moving along with them   */
  const int32_t *wall;       /* [n] (boundary 1; NULL: none) 0 free sphere, 1 bottom-wall
                                sphere, 2 top-wall sphere.  A wall sphere keeps its y and z,
                                moves at its wall's velocity with no spin, and must keep
                                pair_cutoff / 2 from its own face (centre y > a + cutoff/2
                                at the bottom, < ly - a - cutoff/2 at the top)            */
} susp_params;

/* Fill *p with the paper's defaults (tau 1, rho0 1, map_ratio 0.95, rho_p 1, kt 0.5 kn,
 * mu 1, lub_hc 0.5 with subtraction, pair_cutoff 1, n_sub 8, FP32, no shear, BGK with
 * tau_bulk = tau_ghost = 1).                                                             */
void susp_default_params(susp_params *p);

/* Exact device bytes a simulation of these parameters needs (workspace size).  Returns 0
 * and sets the last error if the parameters are invalid.                                  */
size_t susp_footprint_bytes(const susp_params *p);

/* Create a simulation: validate, upload the spheres, fill the fluid with the equilibrium
 * of the imposed shear profile u_x = gdot(0) (y - (ly-1)/2) and map the spheres.
 * Limits (SUSP_EINVAL beyond them): every edge >= 8 nodes; one population array
 * (19 x nodes x storage bytes) < 4 GiB, i.e. up to ~56M nodes in FP32, ~28M in FP64.
 * stream: a hipStream_t (NULL: null stream).  workspace: device memory of at least
 * ws_bytes >= susp_footprint_bytes(p), 256-byte aligned, or NULL to let the library
 * allocate.  On success *out receives the handle.                                         */
int susp_create(const susp_params *p, void *stream, void *workspace, size_t ws_bytes,
                susp_sim **out);

/* Advance nsteps lattice steps (nsteps >= 0).  Returns SUSP_EUNSTABLE if any of those
 * steps found overlapping mapped spheres, a non-finite particle state, a neighbour-list
 * overflow, a node linked to more than six spheres or a sphere displaced by more than one
 * node in one step (the state has still been advanced; after a displacement that large the
 * solid map is no longer updated and the state is meaningless).                            */
int susp_step(susp_sim *s, int64_t nsteps);

/* Stress averaged over the steps since the previous call (or creation), then reset:
 * out[k][c], k = fluid, particle surface, lubrication, contact, DLVO; c = xx yy zz xy xz
 * yz, each divided by the box volume (eqs. 12, 14, 15).  gg = {G', G''} from eqs. (17)-(18)
 * over the observation steps completed so far (0 if none).  Synchronises.                */
int susp_stress(susp_sim *s, double out[5][6], double gg[2]);

/* Health of the run since the previous call (or creation), then reset.  out[0] = fluid
 * node-steps whose speed exceeded 0.3 c_s (past the low-Mach range of the lattice fluid; a
 * node squeezed into a one-node gap between two surfaces passes it briefly in dense runs,
 * so it is counted, not failed), out[1] = the largest |u| / c_s among them (0 if none),
 * out[2] = the relative drift |M + L - M0| / M0 of the fluid mass M plus the ledger L of
 * covered nodes at the last step against its value at the first step (or the last state
 * load).  Synchronises.                                                                    */
int susp_health(susp_sim *s, double out[3]);

/* Walls (boundary 1): mean force per step of the suspension on the bottom and the top wall
 * since the previous call (or creation), then reset.  out[6] (host) = bottom x y z, top
 * x y z: the flat wall (momentum of the bounced populations, measured from the rest state
 * rho0, so that its y part omits the constant rest pressure), plus, for every sphere of the
 * wall, its hydrodynamic force, the substep mean of its pair forces and the momentum of the
 * nodes it covers and releases.  The shear stress on the top wall is out[3] / (lx lz) with
 * the sign of the force on the wall.  SUSP_EINVAL without walls.  Synchronises.           */
int susp_wall_force(susp_sim *s, double out[6]);

/* Contact-force statistics of Sec. 4.2 (eqs. 19-23) and the stress built from them (eq. 27
 * for 3D suspensions, eq. 26 for monolayers; App. C), over the steps since the previous call
 * (or creation), then reset.  Needs contact_bins > 0; nbins must equal it (else SUSP_EINVAL).
 * A contact is a pair whose surfaces overlap at the last DEM substep of a step.  Its
 * orientation theta in [0, pi) is that of the in-plane part (x, y) of the centre-to-centre
 * vector (both senses are one orientation; no in-plane part counts as 0), binned in nbins
 * equal bins.  F_nor: normal contact force, positive when it pushes the spheres apart;
 * F_tan: component along t = (-sin theta, cos theta) of the tangential contact force on the
 * sphere from which n = (cos theta, sin theta) points to the other, positive when it turns
 * that sphere counterclockwise.
 *   hist[5][nbins] (host, caller-owned): per bin centre, rho(theta) normalised as in eq. 23,
 *     xi_N = F_nor(theta) / <F_nor> (eq. 21), xi_T = F_tan(theta) / <F_nor> (eq. 22),
 *     zeta_N = rho xi_N (eq. 19), zeta_T = rho xi_T (eq. 20); F_nor(theta) and F_tan(theta)
 *     are the mean forces of the bin's contacts, <F_nor> the mean over all contacts.
 *   summary[12] (host): samples (steps), contacts per step, Z = 2 contacts / spheres,
 *     <F_nor>, sigma_hat xx, xy, yx, yy (eq. 27 in 3D, eq. 26 per unit volume in a monolayer,
 *     with the integral over the contacts themselves and the prefactor that makes it the
 *     contact virial for equal spheres at distance 2a: 3 phi Z / (4 pi a^2), phi Z / (pi a lz);
 *     compression counts positive), Delta lambda, P, Delta lambda / P of the mean total
 *     stress over the same steps (3D: largest minus smallest eigenvalue and minus the mean
 *     eigenvalue; monolayer: the x-y block), and phi (volume, or area, fraction).
 * Synchronises.                                                                            */
int susp_contact_stats(susp_sim *s, int32_t nbins, double *hist, double summary[12]);

/* susp_contact_stats for callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid allocation): the same read-out, with
 * the final kernel's staging in a static device array that each device holds for the life
 * of the process (at most 180 bins: nbins above that is SUSP_EINVAL) instead of the
 * simulation's own staging.  Calls no allocating routine.  Calls from several host threads
 * are serialised; the array keeps the last call's contents.  Synchronises.                  */
int susp_contact_stats_noalloc(susp_sim *s, int32_t nbins, double *hist, double summary[12]);

/* Release the simulation (and its device block unless it came from a workspace). */
int susp_destroy(susp_sim *s);

/* ---- state access (synchronising); used for checkpoints and parity checks ---- */
/* Populations as full FP64 values n_q, [19][lz][ly][lx]; entries of solid nodes are
 * undefined on get and ignored on set.  Set rounds to the storage precision.  Both stage
 * one plane at a time through the simulation's spare population buffer (the one the next
 * step overwrites) and allocate no device memory.                                         */
int susp_get_populations(susp_sim *s, double *host);
int susp_set_populations(susp_sim *s, const double *host);
/* Running sums of the step's observables, for checkpoints and for checks that start two
 * simulations from one state.  acc[0..29] = stress sums [5][6] (same order as susp_stress)
 * since the previous susp_stress, acc[30] = the number of steps in them, acc[31], acc[32] =
 * the sums of sigma_xy cos(phase) and sigma_xy sin(phase) over the observation steps so far
 * (eqs. 17-18; the phase of eq. 16), acc[33] = their count, acc[34] = the mass ledger: fluid
 * mass taken in by nodes that spheres covered minus the mass given back to released nodes
 * (the fluid mass plus the ledger is conserved while no two spheres touch node to node).  Set checks that every entry is finite and
 * the counts are not negative (SUSP_EINVAL).  Both synchronise.                           */
enum { SUSP_NACC = 35 };
int susp_get_accumulators(susp_sim *s, double acc[SUSP_NACC]);
int susp_set_accumulators(susp_sim *s, const double acc[SUSP_NACC]);
/* The whole state of a simulation in one host buffer, a checkpoint: its step, the populations
 * exactly as stored (deviations from the rest state in the storage type, so a restart is bit
 * for bit in every precision), positions, velocities, spins, orientations, the spring history
 * and the running sums above.  Get: host NULL sets *bytes to the size needed (it varies with
 * the number of pairs in contact); otherwise *bytes must be at least that, and receives it.
 * Set: the buffer must come from a simulation of the same precision, box and sphere count
 * (SUSP_ESTATE otherwise, nothing changed); the caller owns the buffer.  Both synchronise.  */
int susp_get_state(susp_sim *s, void *host, size_t *bytes);
int susp_set_state(susp_sim *s, const void *host, size_t bytes);
/* Particle state: positions, velocities, angular velocities [n][3], orientations [n][4]
 * (any pointer may be NULL on get).  Set re-maps the spheres (no cover/uncover).         */
int susp_get_particles(susp_sim *s, double *pos, double *vel, double *omega, double *quat);
int susp_set_particles(susp_sim *s, const double *pos, const double *vel, const double *omega,
                       const double *quat);
/* Tangential-spring history: the pairs (i<j) in contact and their spring vectors.
 * Get: *count receives the number of pairs; i, j, xi may be NULL to query the count;
 * otherwise they must hold cap entries.  Set replaces the history.                        */
int susp_get_history(susp_sim *s, int32_t cap, int32_t *count, int32_t *i, int32_t *j,
                     double *xi);
int susp_set_history(susp_sim *s, int32_t count, const int32_t *i, const int32_t *j,
                     const double *xi);
/* Step counter and Lees-Edwards offset of the current state; the counter drives eq. (16).
 * Setting the clock re-maps the spheres with the new offset; an overlap this creates is
 * reported by the next susp_set_particles or susp_step, so set the clock first when
 * restoring a state.                                                                     */
int susp_get_clock(susp_sim *s, int64_t *step, double *offset);
int susp_set_clock(susp_sim *s, int64_t step);

/* Per-particle hydrodynamic results of the last step: force [n][3], torque [n][3],
 * symmetric stresslet [n][6] (xx yy zz xy xz yz; link momentum minus that of the uniform
 * rest state) and boundary-link count [n].  Any pointer may be NULL.                      */
int susp_get_hydro(susp_sim *s, double *force, double *torque, double *stresslet,
                   int32_t *nlinks);

/* Lists, for bit-exact checks.  kind selects:
 *   SUSP_LIST_OWNER   int32 [lz][ly][lx] owner sphere of every node (-1 fluid)
 *   SUSP_LIST_GHOST   int32 [2][lz][lx] owner of the ghost points (x,-1,z), (x,ly,z)
 *                     used by the last step
 *   SUSP_LIST_CELLS   int32 cell_start[ncell+1] followed by sphere ids [n] of the cell
 *                     list of the last step (cells x fastest, ids ascending in a cell)
 *   SUSP_LIST_PAIRS   int32 [npairs][2] neighbour pairs (i<j) of the last step, sorted
 *   SUSP_LIST_CONTACTS int32 [m][2] pairs of the last step's list in contact (gap < 0)
 *                     at its start, sorted
 *   SUSP_LIST_LINKS   int32 [nlinks][3] (node, q, sphere) of every link from a fluid
 *                     node whose pull source x - c_q is solid, for the current map and
 *                     offset, sorted by (node, q)
 * *bytes is in/out: capacity of host on entry, bytes needed on return.  host may be NULL
 * to query the size.                                                                       */
enum { SUSP_LIST_OWNER = 0, SUSP_LIST_GHOST = 1, SUSP_LIST_CELLS = 2, SUSP_LIST_PAIRS = 3,
       SUSP_LIST_CONTACTS = 4, SUSP_LIST_LINKS = 5 };
int susp_get_lists(susp_sim *s, int32_t kind, void *host, size_t *bytes);

/* Resolved constants: {m0, kn, kt, eta_n, lub_delta, F0, debye_lambda, eta0, a_min, a_max}. */
int susp_get_derived(susp_sim *s, double out[10]);

/* Graph replay of steps.  On a stream other than the null stream, susp_step records
 * 2 x pairs consecutive steps once as a HIP graph and replays it for every run of that
 * many steps (the buffer parities repeat every two steps; the shear protocol is read from
 * a device table that susp_step uploads ahead of the steps); left-over steps are launched
 * one by one.  Results are bit-identical to plain launches.  pairs in [0, 64], default 5;
 * 0, the null stream or profiling: every kernel is launched one by one.                   */
int susp_use_graphs(susp_sim *s, int32_t pairs);

/* Timing of the lattice step with HIP events on the simulation's stream: while enabled,
 * every step records events around the bounce-back kernel (k_links: the links' bounce-back
 * values and exchanged momentum, eqs. 6-10) and around the streaming kernel (k_stream: pull,
 * collision, fluid stress; eqs. 3-5), the step's dominant kernel.  susp_profile_read
 * synchronises, returns the summed k_stream time in milliseconds and the number of timed
 * steps since the previous read, and resets both; susp_profile_read_parts returns ms[0] =
 * the summed k_links time and ms[1] = the summed k_stream time the same way.               */
int susp_profile(susp_sim *s, int32_t enable);
int susp_profile_read(susp_sim *s, double *ms_total, int64_t *launches);
int susp_profile_read_parts(susp_sim *s, double ms[2], int64_t *launches);

/* ---- Batches: many independent simulations sharing one GPU --------------------------
 * A batch holds up to max_jobs simulations of any box size and parameters, each with its
 * own device block and its own HIP stream (created by the batch, default priority), and
 * admits a new one only while the sum of their susp_footprint_bytes stays within
 * hbm_budget.  susp_batch_step queues the steps of every job on its stream (pairs of steps
 * replayed from one recorded HIP graph per job, see susp_use_graphs), so that small jobs
 * fill the GPU together, then waits for all of them.  A job stepped in a batch gives the
 * same results, bit for bit, as the same job stepped alone.
 * Brick shapes: with autotune set, a job whose brick_y/brick_z are 0 gets the shape that
 * ran its lattice kernel fastest among a few candidates, timed on a scratch copy of the job
 * the first time its (lx, ly, lz, precision, with/without spheres) is seen; the choice is
 * kept for the batch's lifetime.                                                            */
typedef struct susp_batch susp_batch;

/* max_jobs >= 1; hbm_budget in bytes (> 0). */
int susp_batch_create(int32_t max_jobs, size_t hbm_budget, int32_t autotune, susp_batch **out);

/* Admit a job.  On success *slot receives its index (0 <= slot < max_jobs).  SUSP_ENOMEM
 * with nothing changed if its footprint does not fit in the remaining budget, SUSP_ESTATE
 * if every slot is taken; otherwise the errors of susp_create.                              */
int susp_batch_add(susp_batch *b, const susp_params *p, int32_t *slot);

/* Release a job and its device memory (its slot becomes free). */
int susp_batch_remove(susp_batch *b, int32_t slot);

/* Advance every admitted job by nsteps (>= 0).  SUSP_EUNSTABLE if any job reported an
 * instability (the message names the slots; all jobs have still been advanced).           */
int susp_batch_step(susp_batch *b, int64_t nsteps);

/* Queue nsteps steps of one job on its stream and return at once (continuous batching:
 * every job runs as soon as it is queued, none waits for another).  susp_batch_poll sets
 * *done to 1 once the job's queued steps have completed, and then returns its status
 * (SUSP_EUNSTABLE if they raised an instability), else *done = 0 and SUSP_OK.             */
int susp_batch_launch(susp_batch *b, int32_t slot, int64_t nsteps);
int susp_batch_poll(susp_batch *b, int32_t slot, int32_t *done);

/* Queue nsteps steps of every job in the batch in lockstep and return at once (a batched
 * step with one launch per kernel over all jobs; the paper steps one suspension at a time).
 * Jobs whose steps have the same kernel sequence share each kernel's launch: its work-groups
 * are dealt to the jobs by a table of offsets, and each job's arguments come from a device
 * table that the batch builds from the job's own launches.  The jobs are split over four
 * streams by size.  Tables are rebuilt when jobs join or leave; the first run after that
 * issues its kernels one by one, and a run of the same jobs again records one pair of steps
 * of all of them as a HIP graph and replays it.  A run longer than 4096 steps uploads each
 * job's next clock table only after the lockstep work before it.  A job gets exactly the kernels and
 * arguments it would get alone, so its results are the same bit for bit.  Jobs with moving
 * walls, contact statistics, implicit lubrication, profiling, no spheres or a brick other
 * than 64 x 4 x 4 step on their own streams instead.  Waits for the previous lockstep run
 * before it queues anything; an odd step count ends with one step per job on its own stream.
 * susp_batch_poll reports each job as before.  A job's state must not be read
 * (susp_batch_sim getters) before its poll reports it done; susp_batch_stress and
 * susp_batch_remove wait for the run themselves.  Adding a job while a run is in flight is
 * allowed but its creation may wait behind the run (its stream can share a hardware queue
 * with the lockstep streams).
 * Errors: SUSP_EINVAL (NULL batch, negative count), SUSP_ENOMEM (launch tables),
 * SUSP_EDEVICE.                                                                            */
int susp_batch_launch_all(susp_batch *b, int64_t nsteps);

/* susp_stress of one job. */
int susp_batch_stress(susp_batch *b, int32_t slot, double out[5][6], double gg[2]);

/* The job's simulation handle, for the state getters (NULL if the slot is free).  It stays
 * owned by the batch: do not destroy it.                                                   */
susp_sim *susp_batch_sim(susp_batch *b, int32_t slot);

/* Sum of the admitted jobs' footprints, in bytes. */
size_t susp_batch_bytes(const susp_batch *b);

/* The brick shape autotuning gives (or has given) jobs of these parameters. */
int susp_batch_tune(susp_batch *b, const susp_params *p, int32_t *brick_y, int32_t *brick_z);

/* Release every job, the streams and the batch. */
int susp_batch_destroy(susp_batch *b);

/* Text of the calling thread's last error ("" if none). */
const char *susp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
