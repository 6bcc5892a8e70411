// Internal layout shared by the HIP kernels and the host side of libsw.
// Not part of the public ABI (include/sw.h is).
//
// Data layout in HBM (all arrays indexed by the internal atom index i, which
// is the caller's atom order re-sorted per replica along a Morton curve over
// the binning cells, each replica padded to a multiple of 64 atoms):
//   u[2][Npad]        uint4   positions as unsigned 32-bit fractions of the box
//                             edge (x = u * L / 2^32); ping-pong buffers
//   v[Npad], f[Npad]  float4  velocities (A/fs), forces (kcal/mol/A)
//   uref[Npad]        uint4   positions at the last neighbour-row build
//   ids[Npad]         int     caller index of internal atom i (-1 for padding)
//   nl[Npad][cap]     int     neighbour rows (internal indices, ascending)
//   nn[Npad]          int     row lengths
//   act[Npad][cap]    int     with 8 or fewer lanes per atom: the row's entries within the
//                             cutoff at the last moments launch, in row order
//   nact[Npad]        int     their number
//   mom[Npad][3]      float4  per-centre three-body moments and energies
//   gcnt[2][Ctot], gmem[2][Ctot][cc]   binning cells (ping-pong), positions with
//                                      the internal index in .w
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace swk {

constexpr int kBlock = 256;        // threads per block of every atom kernel
constexpr int kRankInts = 16 + 27;  // cell-start mask (8 words + prefix counts) and cell bases of a row rebuild
constexpr int kTile = 64;          // replicas are padded to multiples of this
constexpr int kMaxLPA = 64;        // most lanes per atom of any kernel variant
constexpr int kMinAPB = kBlock / kMaxLPA;   // fewest atoms per block: sizes per-block buffers
constexpr int kNQ = 12;            // thermo quantities per replica
// Row rebuild staging in LDS (moments kernel), per block: candidate and
// sorted rows [2][APB][cap] ints, row counts [APB], per-atom cell prefix and
// cell ids [APB][56].
// LDS of one moments block (apb atoms per block, rows of cap slots): the
// rebuild's candidate and sorted lists, counts, cell prefixes and ids, and
// with 16 or more lanes per atom (apb <= 16) the candidates' positions,
// 16-byte aligned after the int part.
// Per-atom stride (ints) of the rebuild's candidate and sorted lists in LDS.
// With 4 or 8 lanes per atom (apb 64 or 32) it is padded to LPA mod 2 LPA,
// so the groups of a wavefront, each reading LPA consecutive words, start on
// distinct LDS banks (capacity 48 at 8 lanes: stride 56, not 48, whose groups
// g and g + 4 share banks).
__host__ __device__ constexpr int lds_row_stride(int apb, int cap) {
  return apb >= 32 ? cap + ((kBlock / apb) - cap % (2 * (kBlock / apb)) + 2 * (kBlock / apb)) % (2 * (kBlock / apb))
                   : cap;
}
__host__ __device__ constexpr size_t moments_lds_ints(int apb, int cap) {
  return 2 * (size_t)apb * lds_row_stride(apb, cap) + apb + 56 * (size_t)apb;
}
__host__ __device__ constexpr size_t moments_lds_bytes(int apb, int cap) {
  return ((sizeof(int) * moments_lds_ints(apb, cap) + 15) & ~(size_t)15) +
         (apb <= 16 ? 16 * (size_t)apb * cap : 0);
}
constexpr double kAcc = 4.184e-4;  // (A/fs^2) per ((kcal/mol/A)/(g/mol))
constexpr double kBoltz = 8.314462618 / 4184.0;  // kcal/(mol K)
constexpr double kTwo32 = 4294967296.0;
constexpr double kBar = 1e5 * 1e-30 * 6.02214076e23 / 4184.0;   // kcal/mol/A^3 per bar

// Flag slots in Dev::flags.
// Slots below F_REBUILDS are cleared at the start of every call; F_REBUILDS
// counts row rebuilds over the context's lifetime.
enum { F_NBR_OVER = 0, F_NBR_NEED = 1, F_CELL_OVER = 2, F_OVERLAP = 3, F_ABORT = 4, F_BOX = 5, F_PGROUPS = 6,
       F_REBUILDS = 7,
       F_NFLAGS = 8 };

struct RepInfo {
  double L[3];        // box edges (A)
  float scale[3];     // L / 2^32 : fraction units -> A
  float inv_scale[3]; // 2^32 / L
  int nc[3];          // binning cells per edge (each edge >= cutoff + skin)
  int cell_off;       // first cell of this replica in the concatenated grid
  int ncell;
  int ioff;           // first internal atom
  int iend;           // ioff + n
  int ipad_end;       // ioff + roundup(n, 64)
  int n;
  long long uoff;     // first caller atom
  double ndof_kb;     // (3n - 3) k_B
};

// Device pointers and sizes of one context (passed by value to kernels).
struct Dev {
  uint4* u[2];
  float4* v;
  float4* f;
  uint4* uref;
  int* ids;
  int* nl;
  int* nn;
  float4* mom;
  int* gcnt[2];
  uint4* gmem[2];      // [2][Ctot][cc] binned positions, .w = internal index
  double* partial;     // [nblocks][kNQ]
  double* thermo_cur;  // [R][kNQ]
  int* arrive;         // [R]
  int* dflag;          // [2][R] set when an atom of the replica moved > half skin since its build
  int* flags;          // [F_NFLAGS]
  const RepInfo* reps;
  const int* tile_rep; // [Npad / 64] replica of each 64-atom tile
  const double* T0;    // [R] thermostat targets
  const float2* npt_kick;  // [R] (a, b) of the isobaric half kick v <- a v + b F
  double* lref;        // [R] box edge 0 at the replica's last row build
  int npad, cap, cc, ctot, R;
  int max_rep_pad;     // largest padded replica size (atoms)
  // last, so the fields every kernel reads keep their argument offsets
  int* act;            // [Npad][cap] entries within the cutoff (8 or fewer lanes per atom)
  int* nact;           // [Npad]
  int sync_rb;         // every replica rebuilds when any replica's flag is set
};

// Per-call physical constants, pre-folded for the kernels.
struct Phys {
  float rc, rc2;        // a*sigma and its square
  float rl2;            // (cutoff + skin)^2 : row radius
  float half_skin;      // rebuild when an atom moved more than this (A)
  float sig, sig_l2e;   // sigma, sigma*log2(e)
  float gsig, gsig_l2e; // gamma*sigma and times log2(e)
  float Aeps, B;        // A*epsilon, B
  float lameps, c0, qc; // lambda*epsilon, cos(theta0), (1 - cos theta0)^2
  float hdt_cm;         // dt/2 * 4.184e-4 / mass
  float dt;
  float half_m_acc;     // 0.5 * mass / 4.184e-4 (KE in kcal/mol from A/fs)
  float m_acc;          // mass / 4.184e-4
  double dt_d, tau_d;   // thermostat
  int thermostat;       // SW_NVE / SW_RESCALE / SW_BERENDSEN
  float term2, term3;   // weights of the two- and three-body terms in a tangent pass (sw_grad's
                        // term mask; 1 elsewhere)
};

// Kernel modes of the force kernel.
enum { MODE_FORCES = 0, MODE_START = 1, MODE_NVE = 2, MODE_NVE_LAST = 3, MODE_KICK = 4, MODE_NPT = 5 };

// Isothermal-isobaric dynamics (Nose-Hoover chains on the particles and on
// an isotropic barostat).  One replica's extended variables, FP64.
constexpr int kNptChain = 4;
struct NptState {
  double L[3];                             // box edges (A)
  double ve;                               // barostat rate v_e (1/fs)
  double xi[kNptChain], vxi[kNptChain];    // particle chain
  double eta[kNptChain], veta[kNptChain];  // barostat chain
};
enum { NPT_BEGIN = 1, NPT_STEP = 3, NPT_END = 2 };   // bit 1: open a step, bit 2: close the previous one
// Per-replica constants of the extended system, fixed for one call (made on
// the host from the target temperature, the relaxation times and the atom
// count): the device chain arithmetic then has no division.
struct NptConst {
  double nf, kT, alpha;                    // particle degrees of freedom, k_B T0, 1 + 3 / nf
  double Q[kNptChain], iQ[kNptChain];      // particle chain masses and their reciprocals
  double Qb, iQb;                          // barostat chain mass (every link) and reciprocal
  double Wb, iWb;                          // barostat mass and reciprocal
  double pext;                             // external pressure (kcal/mol/A^3); 0 without barostat
};
struct NptArgs {
  const NptState* in;    // [R] state before this launch
  NptState* out;         // [R] state after it
  RepInfo* reps;         // writable view: box edges and scales follow the state
  float2* kick;          // [R] kick coefficients of the step opened here
  const NptConst* cst;   // [R]
  double tauT, tauP, rl, rc, dt, c_m;
  int chain;             // chain length 1..kNptChain
  int apb;               // atoms per block of the force launch: replicas of at most
                         // kFusedBlocks such blocks sum its block partials here,
                         // larger ones read the reduction launch's thermo_cur
  int mode;              // NPT_BEGIN / NPT_STEP / NPT_END
  int par;               // parity of the positions this launch reads
  double* row;           // [R][kNptRow] record of the step closed here, or null
};
constexpr int kNptRow = 11;
// Largest count of force blocks per replica whose partials the kernel after
// the force launch (isobaric kick, thermostat) sums in every wave of the
// replica (the work grows with the square of the replica size; larger
// replicas take their sums from a reduction launch).
constexpr int kFusedBlocks = 512;
// Whether some replica of d is too large for those in-kernel sums at apb
// atoms per force block.
__host__ __device__ inline bool needs_reduce_launch(const Dev& d, int apb) {
  return d.max_rep_pad / apb > kFusedBlocks;
}

// Optional start/stop events recorded at a launch's dispatch.
struct KTimer {
  hipEvent_t start = nullptr, stop = nullptr;
};

// Host launchers (sw_kernels.hip).  Each returns a hipError_t.
hipError_t launch_sort(const Dev& d, const float4* x_user, const float4* v_user, long long n_user,
                       const long long* uoff, int R, const int* cell_rank, uint4* uq, int* key,
                       int* cnt, int* start, int* cursor, int* order, hipStream_t s);
hipError_t launch_gather_ids(const Dev& d, const float4* x_user, int par, hipStream_t s);
// Bins u[par] into grid par; with check_disp, flags replicas with an atom too far from its
// row-build position for rows of radius rl (in the box of the build) to cover rc.
hipError_t launch_bin(const Dev& d, int par, int check_disp, float rl, float rc, hipStream_t s);
hipError_t launch_moments(const Dev& d, const Phys& p, int lpa, int par, int force_rebuild,
                          int energy, hipStream_t s, const KTimer& tm = KTimer());
hipError_t launch_forces(const Dev& d, const Phys& p, int lpa, int mode, int vir, int par,
                         double* ring_row, hipStream_t s, const KTimer& tm = KTimer());
// Moments with energies at parity par and, in the same launch, their tangent
// along w (mdot [Npad][3]); rows rebuilt if forced or flagged.
hipError_t launch_moments_tan(const Dev& d, const Phys& p, int lpa, int par, int force_rebuild, const float4* w,
                              float4* mdot, hipStream_t s);
hipError_t launch_thermostat(const Dev& d, const Phys& p, int lpa, int par, int last, hipStream_t s);
// Audit of the rows in use at parity par against a fresh search of grid par:
// counts[0] += pairs closer than the cut-off, counts[1] += those missing from
// their row.
hipError_t launch_audit(const Dev& d, const Phys& p, int par, unsigned long long* counts, hipStream_t s);
hipError_t launch_scatter_out(const Dev& d, int par, float4* x_user, float4* v_user,
                              float4* f_user, hipStream_t s);
hipError_t launch_copy_thermo(const Dev& d, double* energy, double* virial, hipStream_t s);
hipError_t launch_fill_i32(int* p, int value, long long n, hipStream_t s);
hipError_t launch_fill_f32(float* p, float value, long long n, hipStream_t s);
hipError_t launch_fill_f64(double* p, double value, long long n, hipStream_t s);
hipError_t launch_npt_kick(const Dev& d, const Phys& p, const NptArgs& a, hipStream_t s);

// Persistent cooperative launch of steps t0..t1 of an sw_step call.
struct PArgs {
  int t0, t1;          // first and last step of this launch (t1 - t0 < kPersistSteps)
  int nsteps;          // steps of the whole call (the last one ends on a full-step velocity)
  int thermo_every;    // 0 = no thermo rows
  int rebuild_every;   // forced row rebuild period (0 = none)
  double* thermo;      // caller table [nsteps / thermo_every][R][kNQ] or null
  unsigned* ctl;       // [kCtlWords] control words (zeroed by the launcher)
  int* abort;          // raised by a barrier wait that timed out (flags[F_ABORT])
  int sync_rb;         // synchronised rebuilds (the kernel gets Dev::sync_rb = 0)
  int ng;              // replica groups (1: grid-wide barriers)
  unsigned xmask;      // XCC ids of the groups, one bit each (ng bits set)
  const int* gtab;     // group table (layout below), ng > 1
};
// Control words of a persistent launch.  Words that many blocks add to or
// poll sit 64 words (256 B) apart.
constexpr int kMaxXcc = 16;                      // XCC ids are 4 bits
constexpr int kPersistSteps = 4096;              // steps of one launch
constexpr int kCtlGrid = 0;                      // arrivals at grid-wide barriers
constexpr int kCtlGroup = 64;                    // + 64 x: arrivals at the barriers of XCC x
constexpr int kCtlCensus = 64 * (1 + kMaxXcc);   // + x: blocks found on XCC x
constexpr int kCtlStep = kCtlCensus + 64;        // + s: step t0 + s done by a group (low byte),
                                                 //   rebuild flags raised (<< 8)
constexpr int kCtlEpoch = kCtlStep + kPersistSteps;   // + 256 x + cu: last barrier whose L1
                                                      //   invalidate a block of that CU took on
constexpr int kCtlDone = kCtlEpoch + kMaxXcc * 256;   // + 256 x + cu: last barrier whose
                                                      //   invalidate is done
constexpr int kCtlWords = kCtlDone + kMaxXcc * 256;
// Group table of the persistent launch (ints): offsets [ng + 1] of the
// groups' padded atoms in 64-atom units, offsets [ng + 1] into the replica
// list, then the replicas of group 0, 1, ... in ascending order.
hipError_t launch_persistent(const Dev& d, const Phys& p, int lpa, const PArgs& a, int blocks_per_cu,
                             hipStream_t s, int* grid_out);
// Bit mask of the XCC ids the device's compute units report.
hipError_t xcc_census(unsigned* d_word, unsigned* mask_out, hipStream_t s);

// Tangent (forward-mode) kernels for sw_grad / sw_adjoint.
constexpr int kTQ = 8;  // per replica: E2, E3, W2 trace, W3 trace, w.F, w.F3, d(W trace) along w,
                        // d(W trace)/ds under a uniform scaling of every leg (adjoint virial term)
struct Tan {
  float4* w;         // [Npad] tangent direction (A), internal order
  float4* mdot;      // [Npad][3] tangent of the moments
  float4* fdot;      // [Npad] tangent of the forces: (dF/dx) w
  float4* f3;        // [Npad] three-body part of the forces
  float4* gw;        // [Npad] gradient of the virial trace, F + dF/ds (adjoint virial term)
  double* tpartial;  // [kTQ][nblocks]
  double* tsum;      // [R][kTQ]
};
// Per-frame adjoint update fused into the tangent force kernel.
struct Adj {
  float4* xb;        // [Npad] position adjoint, updated in place
  float4* vb_next;   // [Npad] next direction vb + dt xb (unused on the last frame)
  float coef_cm;     // frame weight (dt or dt/2) * 4.184e-4 / mass
  float dt;
  float aU, a3;      // loss weights
  int S;             // trajectory steps (loss normalisation 1 / (n_r (S + 1)))
  int last;          // last frame: do not form the next direction
  double coef_d;     // the frame weight coef_cm in double, applied to the w.F sums below
  double* tacc;      // [kTQ][nblocks] per-block sums over the sweep's frames (w.F terms
                     // weighted by coef_d); one reduction after the sweep
  const uint4* unext;  // positions of the frame the sweep visits next, or null: an atom
                       // more than half the skin from its row-build position raises the
                       // replica's flag of the other parity (that frame rebuilds its rows)
  float aW;            // weight of the virial trace in the loss
  const float4* gw;    // [Npad] this frame's virial gradient (read when aW != 0)
};
hipError_t launch_gather_vec(const Dev& d, const float4* user, float4* internal, hipStream_t s);
hipError_t launch_scatter_vec(const Dev& d, const float4* internal, float4* user, hipStream_t s);
hipError_t launch_copy_u(const Dev& d, const uint4* src, uint4* dst, hipStream_t s);
hipError_t launch_copy_v(const Dev& d, const float4* src, float4* dst, hipStream_t s);

}  // namespace swk
