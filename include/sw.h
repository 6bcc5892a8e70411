/*
 * sw.h - C ABI of the mW Stillinger-Weber molecular-dynamics engine for
 * AMD MI355X (gfx950).
 *
 * The model (Molinero & Moore, "Water modeled as an intermediate element
 * between carbon and silicon", Sec. II.A, the equations for E, phi2 and phi3):
 *
 *   E = sum_i sum_{j>i} phi2(r_ij) + sum_i sum_{j!=i} sum_{k>j,k!=i} phi3(r_ij, r_ik, theta_jik)
 *   phi2(r)     = A eps [B (sig/r)^p - (sig/r)^q] exp(sig / (r - a sig))
 *   phi3(r,s,t) = lam eps (cos t - cos t0)^2 exp(gam sig/(r - a sig)) exp(gam sig/(s - a sig))
 *
 * with every term zero beyond the reduced cut-off a*sig, the vertex of
 * theta_jik at atom i, and the mW parameters of Sec. II.D (lam = 23.15,
 * eps = 6.189 kcal/mol, sig = 2.3925 A; A, B, p = 4, q = 0, gam = 1.2, a = 1.8
 * from Sec. II.A; cos t0 = -1/3).  Time integration is velocity Verlet; the
 * paper's production step is 10 fs (Sec. II.B).
 *
 * Units: Angstrom, fs, kcal/mol, g/mol, K.  Acceleration a = 4.184e-4 F / m.
 *
 * Conventions shared by every call:
 *  - All array arguments documented as "device" are device pointers owned by
 *    the caller; the library never frees them.  "host" pointers are read
 *    during the call only.
 *  - Atom arrays x, v, f are float[N][4] (x, y, z, w); w is ignored on input
 *    and written as 0 on output.  N = offsets[R] is the total over replicas;
 *    replica r owns atoms offsets[r] .. offsets[r+1]-1.  Atom order in every
 *    caller array is the caller's own: the library keeps its own spatially
 *    sorted copy internally and scatters results back.
 *  - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *    All work is enqueued on it.  Calls that report device-side error flags
 *    (overflow, overlap) synchronise the stream before returning.
 *  - Return values are sw_status codes (0 = success, negative = error).  No
 *    exception crosses the ABI.  One context must not be used from two host
 *    threads at once.
 */
#ifndef SW_H
#define SW_H

#ifdef __cplusplus
extern "C" {
#endif

/* Parameter block, Sec. II.A (A, B, p, q, gamma, a, theta0) and Sec. II.D
 * (lambda, epsilon, sigma).  The GPU kernels implement the Stillinger-Weber
 * exponents p = 4, q = 0; other values return SW_EUNSUPPORTED. */
typedef struct sw_params {
  double lambda;      /* three-body strength                         */
  double epsilon;     /* energy scale, kcal/mol                      */
  double sigma;       /* length scale, Angstrom                      */
  double A, B;        /* two-body form constants                     */
  double p, q;        /* two-body exponents                          */
  double gamma;       /* three-body radial decay                     */
  double a;           /* reduced cut-off: every term vanishes at a*sigma */
  double cos_theta0;  /* cosine of the favoured angle                */
} sw_params;

typedef enum sw_status {
  SW_OK = 0,
  SW_EINVAL = -1,          /* bad argument (NULL pointer, size, value)                 */
  SW_EBOX_TOO_SMALL = -2,  /* a box edge holds fewer than 3 cells of cutoff + skin     */
  SW_ENBR_OVERFLOW = -3,   /* a neighbour row exceeded the capacity even after growth  */
  SW_ECELL_OVERFLOW = -4,  /* a binning cell exceeded its capacity even after growth   */
  SW_EOVERLAP = -5,        /* two atoms closer than 0.5 A, a NaN, or a step moving an
                              atom by more than a quarter box edge                     */
  SW_EHIP = -6,            /* a HIP runtime call failed (see sw_last_hip_error)         */
  SW_ENOMEM = -7,          /* device allocation failed                                 */
  SW_EUNSUPPORTED = -8,    /* parameter or option outside what the kernels implement  */
  SW_ESTATE = -9,          /* call needs state the context does not have              */
  SW_ETIMEOUT = -10,       /* a grid barrier of the persistent launch waited too long  */
  SW_ESCRATCH = -11        /* input too large for sw_forces_noalloc's static scratch   */
} sw_status;

/* Opaque context: replica layout, cell grids, neighbour rows, workspaces. */
typedef struct sw_ctx sw_ctx;

/* Fills *out with the mW parameters (Sec. II.A constants, Sec. II.D values). */
void sw_params_mw(sw_params* out);

/* Creates a context for n_replicas independent periodic orthorhombic boxes.
 *  h_offsets   host, int64[n_replicas+1], offsets[0] = 0, non-decreasing; every
 *              replica holds at least 2 atoms.
 *  h_box       host, double[n_replicas][3], box edges in Angstrom.
 *  cutoff      largest a*sigma any later call may use (Angstrom, > 0).
 *  skin        Verlet skin (Angstrom, >= 0).  Neighbour rows hold every atom
 *              within cutoff + skin; rows are rebuilt when some atom has moved
 *              more than half of (cutoff + skin - a*sigma) since the last build.
 *  nbr_capacity initial slots per neighbour row (grown automatically, <= 512).
 * Errors: SW_EINVAL, SW_EBOX_TOO_SMALL (an edge shorter than 3 (cutoff + skin)),
 * SW_ENOMEM, SW_EHIP.  On success *out owns device memory until sw_destroy. */
int sw_create(sw_ctx** out, int n_replicas, const long long* h_offsets, const double* h_box,
              double cutoff, double skin, int nbr_capacity);

/* Releases everything the context owns.  NULL is ignored. */
void sw_destroy(sw_ctx* ctx);

/* Neighbour search (cell binning, Morton-ordered counting sort, Verlet rows).
 * The paper's cut-off a*sigma (Sec. II.A) bounds the interaction range; the
 * rows list every j != i within cutoff + skin.
 *  x      device float[N][4] positions (any values; wrapped into the box).
 * After this call the context holds a spatial order and rows for x; sw_forces
 * reuses them while they stay valid.  Synchronises; returns SW_ENBR_OVERFLOW /
 * SW_ECELL_OVERFLOW only if growth failed. */
int sw_build_neighbors(sw_ctx* ctx, const float* x, void* stream);

/* Copies the current rows out, in the caller's atom order.
 *  h_counts host int[N]; h_rows host int[N][max_per_row] (caller atom indices,
 *  each row ascending; unused slots set to -1).  Returns SW_EINVAL if a row
 *  is longer than max_per_row, SW_ESTATE before any build. */
int sw_get_neighbors(sw_ctx* ctx, int* h_counts, int* h_rows, int max_per_row);

/* Energy, forces and virial of Eq. E (Sec. II.A) at positions x.
 *  x       device float[N][4].
 *  params  host; p must be 4, q 0, a*sigma <= the context's cutoff.
 *  f       device float[N][4] out: -dE/dx, kcal/mol/A.
 *  energy  device double[R][2] out (may be NULL): E2, E3 per replica, kcal/mol.
 *  virial  device double[R][6] out (may be NULL): W_xx, yy, zz, xy, xz, yz with
 *          W_ab = sum over terms of sum over legs d_a F_b, kcal/mol.
 * Rebuilds rows first when x has moved too far from the last build.
 * Synchronises. */
int sw_forces(sw_ctx* ctx, const float* x, const sw_params* params, float* f, double* energy,
              double* virial, void* stream);

/* Allocation-free variant of sw_forces, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  It needs no context: one periodic box of n atoms is
 * sorted, binned, given rows (cutoff a*sigma + SW_NOALLOC_SKIN) and evaluated
 * with the same kernels as sw_forces, and every device buffer of that work
 * lies in one static device array of SW_SCRATCH_BYTES that each GPU the
 * library runs on holds until the process ends.  Calls allocate and free
 * nothing (host or device side of HIP); they share the array of their GPU,
 * which keeps the last call's contents (each call clears what must start at
 * zero), so calls that overlap on one GPU race.
 *  x       device float[n][4] positions (A), caller order.
 *  n       atoms, 2 <= n <= SW_NOALLOC_MAX_ATOMS (else SW_ESCRATCH).
 *  h_box   host double[3] box edges (A), each at least 3 (a*sigma + skin).
 *  params  host; as for sw_forces (p = 4, q = 0).
 *  f, energy, virial  device outputs as for sw_forces (R = 1).
 * Errors: SW_EINVAL, SW_EBOX_TOO_SMALL, SW_ESCRATCH (the box needs more
 * working memory than the array holds), SW_ENBR_OVERFLOW / SW_ECELL_OVERFLOW
 * (rows hold 64 slots and never grow here), SW_EOVERLAP, SW_EHIP.
 * Synchronises. */
#define SW_SCRATCH_BYTES (32u << 20)
#define SW_NOALLOC_MAX_ATOMS 16384
#define SW_NOALLOC_SKIN 0.5
int sw_forces_noalloc(const float* x, long long n, const double* h_box, const sw_params* params,
                      float* f, double* energy, double* virial, void* stream);

/* Thermostat kinds for sw_step. */
enum { SW_NVE = 0, SW_RESCALE = 1, SW_BERENDSEN = 2 };

/* Width of one thermo record per replica (doubles). */
#define SW_THERMO_WIDTH 12

/* nsteps steps of velocity Verlet (kick-drift-kick) from (x, v):
 *   v += dt/2 a(x);  x += dt v;  v += dt/2 a(x);  then the thermostat
 * with a = 4.184e-4 F / mass.  Thermostats act on the full-step velocities:
 * SW_RESCALE multiplies v by sqrt(T0/T); SW_BERENDSEN by
 * sqrt(1 + dt/tau (T0/T - 1)); T = 2 KE / ((3N_r - 3) k_B) per replica.
 *  x, v    device float[N][4] in/out (A, A/fs).
 *  f       device float[N][4] out: forces at the final positions.
 *  mass    g/mol (> 0); dt fs (> 0); nsteps >= 0.
 *  h_T0    host double[R] target temperatures (K); required unless SW_NVE.
 *  tau_fs  Berendsen time constant (fs).
 *  thermo  device double[nsteps / thermo_every][R][SW_THERMO_WIDTH] out, may
 *          be NULL: for each recorded step (every thermo_every-th step) and
 *          replica: E2, E3, KE (before the thermostat), W xx yy zz xy xz yz,
 *          K xx yy zz (K_aa = sum m v_a^2 in kcal/mol).
 * Synchronises at the end to report device-side flags; on a neighbour or
 * cell overflow the capacity is grown and the whole call is redone from the
 * untouched inputs. */
int sw_step(sw_ctx* ctx, float* x, float* v, float* f, const sw_params* params, double mass,
            double dt, int nsteps, int thermostat, const double* h_T0, double tau_fs,
            double* thermo, int thermo_every, void* stream);

/* Terms of Eq. E (Sec. II.A) selected by sw_grad's term_mask. */
enum { SW_TERM_TWO_BODY = 1, SW_TERM_THREE_BODY = 2 };

/* Tangent of the force field along w at positions x (forward mode):
 *  w         device float[N][4] direction (A).
 *  term_mask SW_TERM_TWO_BODY, SW_TERM_THREE_BODY or both (3): the terms of
 *            Eq. E whose forces, energies and virial enter every output
 *            (other values: SW_EINVAL).
 *  hvp       device float[N][4] out: (dF/dx) w = -H w of the selected terms (H
 *            is symmetric, so this is also (dF/dx)^T w).
 *  wdF       device double[R][3] out (may be NULL): w . dF/d(lambda, epsilon, sigma).
 *  dU        device double[R][3] out (may be NULL): dU/d(lambda, epsilon, sigma).
 * Uses the reduced form of Sec. II.A, which holds for each term on its own:
 * dF/deps = F/eps, dF/dlambda = F3/lambda, dF/dsigma = -(1/sigma) dW/dx with W
 * the virial trace (dU/dsigma = W/sigma). Synchronises. */
int sw_grad(sw_ctx* ctx, const float* x, const float* w, const sw_params* params, int term_mask,
            float* hvp, double* wdF, double* dU, void* stream);

/* Gradient of a trajectory observable by the discrete adjoint of NVE velocity
 * Verlet, with checkpoints every ckpt_every steps and recomputation:
 *   L_r = 1/(S+1) sum_{s=0..S} [aU U_r(x_s) + a3 U3_r(x_s) + aW W_r(x_s)] / N_r
 *         + xbar_S . x_S + vbar_S . v_S
 * (U = E2 + E3, U3 = E3, W the virial trace (the configurational part of
 * the pressure, P V = (2 KE + W)/3, used with the density of Sec. II.D to
 * fix sigma), S = nsteps).  aW != 0 adds one scaling tangent pass per frame
 * (dW/dx and dW/dsigma follow from the reduced form of Sec. II.A).
 *  x0, v0   device float[N][4] initial state (unchanged).
 *  xbar_S, vbar_S device float[N][4] terminal seeds, may be NULL (= 0).
 *  loss     device double[R] out.
 *  xbar0, vbar0 device float[N][4] out: dL/dx0, dL/dv0.
 *  thbar    device double[R][3] out: dL/d(lambda, epsilon, sigma).
 *  xS, vS   device float[N][4] out (may be NULL): final state.
 * Work buffers (a checkpoint per segment, ckpt_every + 1 frames of positions
 * and cells, adjoint vectors) are device memory the context allocates on
 * first use, keeps for later calls (grown when a call needs more) and frees
 * in sw_destroy.  Synchronises once, at the end (a row or cell overflow is
 * found there and the call reruns itself with grown capacities). */
int sw_adjoint(sw_ctx* ctx, const float* x0, const float* v0, const sw_params* params,
               double mass, double dt, int nsteps, int ckpt_every, double aU, double a3,
               double aW, const float* xbar_S, const float* vbar_S, double* loss, float* xbar0,
               float* vbar0, double* thbar, float* xS, float* vS, void* stream);

/* Structural observables (Sec. II.C).  Positions x are the caller's device
 * float[N][4] in A; they are re-sorted into the context's internal order and
 * binned (the context's next sw_step sorts again).  Coordinates follow the
 * engine's convention u = floor(frac(x / L) 2^32) per component, and every
 * distance and angle is formed in FP64 from them with single correctly
 * rounded operations in a fixed order, so the counts are exact functions of
 * x and of the caller's edges.  The search radius is limited to the smallest
 * binning-cell edge, floor-divided from the box by cutoff + skin (the 27
 * surrounding cells are searched).  Synchronise. */

/* Pair distance histogram for g(r) and n_c:
 *  h_r2_edges  host double[nbins + 1], strictly ascending squared distances
 *              (A^2), e[0] >= 0 and e[nbins] <= (smallest cell edge)^2.
 *  counts      device unsigned long long[R][nbins] out: ordered pairs (i, j),
 *              j != i, of replica r with e[0] <= r^2 < e[nbins], in the bin given
 *              by how many of the interior edges e[1..nbins-1] are <= r^2.
 *  1 <= nbins <= 8192.  SW_EINVAL on bad edges or sizes. */
int sw_rdf(sw_ctx* ctx, const float* x, int nbins, const double* h_r2_edges,
           unsigned long long* counts, void* stream);

/* Angular distribution P(theta) over each molecule's n_near closest neighbours
 * (Sec. II.C uses n_c = 8): for every centre k, the neighbours with
 * r^2 < r_search^2 ordered by (r^2, caller index); every unordered pair (a, b)
 * of the first n_near gives cos = (d_a . d_b) / sqrt(r_a^2 r_b^2).
 *  h_cos_edges host double[nbins + 1], strictly descending cosines (ascending
 *              angles); the bin is the number of interior edges
 *              c[1..nbins-1] that are >= cos.
 *  counts      device unsigned long long[R][nbins] out.
 *  h_short     host long long out (may be NULL): centres with fewer than n_near
 *              neighbours inside r_search (skipped).
 *  2 <= n_near <= 16, 0 < r_search <= smallest cell edge.  SW_ENBR_OVERFLOW if
 *  a centre has more than 64 neighbours inside r_search. */
int sw_adf(sw_ctx* ctx, const float* x, int n_near, double r_search, int nbins,
           const double* h_cos_edges, unsigned long long* counts, long long* h_short,
           void* stream);

/* Mean square displacement for the Einstein relation D = lim <|r(t) - r(0)|^2>/6t
 * (Sec. II.C).  The context keeps, in caller order, each atom's position at
 * the last call and its displacement since the reference call, accumulated
 * in FP64 from minimum images (so successive calls must be less than half a
 * box edge of motion apart).
 *  x      device float[N][4] caller order (A).
 *  reset  nonzero: this call is the reference (displacements zeroed).
 *  msd    device double[R] out: per-replica mean of |displacement|^2 (A^2).
 *  SW_ESTATE if the first call does not reset. */
int sw_msd(sw_ctx* ctx, const float* x, int reset, double* msd, void* stream);

/* Isothermal-isobaric dynamics: the Nose-Hoover thermostat and barostat of
 * Sec. II.B (relaxation times tau_T = 1 ps and tau_P = 2.5 ps in the paper,
 * p = 0), read as the isotropic Martyna-Tobias-Klein equations with
 * Nose-Hoover chains of length `chain` on the particles (xi) and on the
 * barostat (eta).  With N_f = 3N_r - 3, kT = k_B T0_r, the masses are
 * Q_1 = N_f kT tau_T^2, Q_k = kT tau_T^2, W = (N_f + 3) kT tau_P^2 and
 * Q'_k = kT tau_P^2.  One step of length dt is the symmetric splitting
 *   chain(eta) chain(xi) barostat kick drift kick barostat chain(xi) chain(eta)
 * (half steps except the drift), exact flows for the kicks
 * v <- v e^{-c h} + h a e^{-c h/2} sinh(c h/2)/(c h/2), c = (1 + 3/N_f) v_e, and
 * the drift, which scales every box edge by e^{v_e dt}.  Every replica has
 * its own box, T0 and pressure; the boxes persist in the context (sw_get_box)
 * and so do the extended variables (sw_npt_state) between calls.
 *  x, v, f   as for sw_step (positions in A in the box at the end).
 *  h_T0      host double[R] K;  h_p_bar host double[R] bar.
 *  chain     1..4 (the paper names no chain length; 3 is customary).
 *  reset     nonzero: extended variables start from zero (box kept).
 *  tau_P_fs  barostat relaxation time; <= 0 turns the barostat off (fixed
 *            box: Nose-Hoover NVT, as for the paper's slab runs).
 *  rows      device double[nsteps / every][R][SW_NPT_WIDTH] out, may be NULL:
 *            after each recorded step: V (A^3), P_int (bar), T (K), U, KE,
 *            p V, extended energy, conserved H' (kcal/mol), then the
 *            pressure tensor diagonal P_xx, P_yy, P_zz (bar).
 * Cell grids are rebuilt with a margin when a box shrinks toward its
 * cutoff + skin edge; the call is then redone from its inputs.
 * Synchronises. */
#define SW_NPT_WIDTH 11
#define SW_NPT_STATE 17   /* v_e, xi[4], vxi[4], eta[4], veta[4] per replica */
int sw_npt(sw_ctx* ctx, float* x, float* v, float* f, const sw_params* params, double mass,
           double dt, int nsteps, const double* h_T0, const double* h_p_bar, double tau_T_fs,
           double tau_P_fs, int chain, int reset, double* rows, int every, void* stream);
/* Current box edges: host double[R][3] out (A). */
int sw_get_box(const sw_ctx* ctx, double* h_box);
/* Extended variables of sw_npt: host double[R][SW_NPT_STATE]; set = 0 reads
 * them, set != 0 replaces them (the box is not part of this state). */
int sw_npt_state(sw_ctx* ctx, double* h_state, int set);

/* Execution options (chosen by the autotuner). */
typedef struct sw_tuning {
  int lanes_per_atom;   /* 4, 8, 16, 32 or 64 lanes of a wavefront per atom   */
  int graph_steps;      /* sw_step and sw_npt replay captured hipGraph blocks of
                           at least this many steps (rounded up to a multiple
                           of 2 and of the record interval); any value > 0 also
                           makes sw_adjoint capture its forward and reverse
                           sweeps on the first call of a configuration and
                           replay them on later calls; with `persistent`,
                           sw_step captures a call's persistent launches and
                           replays them on later calls of the same step count
                           and settings; 0 = plain launches.
                           Results are the same bits either way.               */
  int persistent;       /* 0: one launch per phase; 1: sw_step's steps run in
                           cooperative persistent launches (up to 4096 steps
                           each) at full occupancy; k > 1: the same with at most
                           k blocks per CU.  When the replicas can be dealt to
                           the device's XCCs within 25 % of an even load, each
                           XCC's blocks run its replicas and synchronise among
                           themselves (SW_Q_PERSISTENT_GROUPS); else grid-wide
                           barriers.  Setting it plans the groups (synchronous,
                           allocates the launch's control words).              */
  int rebuild_every;    /* also rebuild rows at least this often (0 = only on
                           displacement)                                        */
  int timing;           /* > 0: every timing-th step of sw_step, bracket the
                           moments and force launches with HIP events and add
                           their durations to the SW_Q_TIME_* counters (an odd
                           period samples steps of both parities, so rebuild
                           steps are sampled at their own rate)                 */
  int sync_rebuild;     /* 1: when any replica's displacement check fires, every
                           replica rebuilds its rows (fewer launches pay for a
                           rebuild when many replicas share a context; a
                           replica then no longer equals the same replica run
                           alone bit for bit, only within rounding); 0: each
                           replica rebuilds on its own check                   */
  int audit_every;      /* > 0: after the moments launch of every audit_every-th
                           step of sw_step (per-phase or captured launches; the
                           persistent launch is not audited), check the rows in
                           use against a fresh search of the binning cells:
                           every pair closer than a*sigma is counted, and so is
                           every such pair missing from its row
                           (SW_Q_AUDIT_PAIRS, SW_Q_MISSED_PAIRS; results are
                           unchanged); 0 = off                                  */
} sw_tuning;
int sw_set_tuning(sw_ctx* ctx, const sw_tuning* t);
int sw_get_tuning(const sw_ctx* ctx, sw_tuning* t);

/* Queries (value written to *out). */
enum {
  SW_Q_NATOMS = 0,        /* total atoms N                             */
  SW_Q_NREPLICAS = 1,
  SW_Q_NBR_CAPACITY = 2,  /* current slots per row                     */
  SW_Q_REBUILDS = 3,      /* row rebuilds since creation               */
  SW_Q_CELL_CAPACITY = 5,
  SW_Q_DEVICE_BYTES = 6,  /* device memory owned by the context        */
  SW_Q_STEPS = 7,         /* integration steps since creation          */
  SW_Q_MIN_CELL_EDGE = 11, /* smallest binning-cell edge in 1e-6 A (the
                              observables' search-radius limit)            */
  SW_Q_TIME_MOMENTS_NS = 8, /* summed event time of sampled moments launches */
  SW_Q_TIME_FORCES_NS = 9,  /* summed event time of sampled force launches   */
  SW_Q_TIMED_STEPS = 10,    /* number of sampled steps (reset by sw_set_tuning) */
  SW_Q_AUDIT_PAIRS = 12,    /* pairs closer than a*sigma seen by audits (sw_tuning.audit_every),
                               since creation                                    */
  SW_Q_MISSED_PAIRS = 13,   /* of those, pairs absent from the rows in use (0 unless the
                               rebuild criterion failed)                         */
  SW_Q_PERSISTENT_GROUPS = 14 /* barrier groups of the last persistent sw_step call:
                               1 = grid-wide barriers, k > 1 = replicas dealt to k XCCs,
                               each group's barriers kept on its XCC; 0 = none yet */
};
int sw_query(sw_ctx* ctx, int what, long long* out);

const char* sw_status_string(int status);
int sw_last_hip_error(const sw_ctx* ctx);   /* hipError_t of the last SW_EHIP */

#ifdef __cplusplus
}
#endif
#endif /* SW_H */
