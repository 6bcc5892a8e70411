// Host-side context of libsw, shared by sw_api.hip and sw_tangent.hip.
#pragma once
#include "sw.h"
#include "sw_internal.h"

#include <algorithm>
#include <unordered_map>
#include <vector>

using swk::RepInfo;
using swk::Dev;
using swk::Tan;

struct sw_ctx {
  int R = 0;
  long long N = 0;
  int npad = 0;
  std::vector<long long> uoff;
  std::vector<double> box;
  double cutoff = 0.0, skin = 0.0;
  int cap = 0, cc = 32;
  std::vector<RepInfo> reps;
  int ctot = 0;
  std::vector<int> tile_rep, cell_rank;
  sw_tuning tune{8, 0, 0, 0, 0, 0, 0};
  std::vector<hipEvent_t> tev;     // sampled launch timing: 4 events per sample
  double t_mom_ms = 0.0, t_for_ms = 0.0;
  long long t_samples = 0;
  Dev d{};
  RepInfo* d_reps = nullptr;
  int* d_tile_rep = nullptr;
  long long* d_uoff = nullptr;
  int* d_cell_rank = nullptr;
  double* d_T0 = nullptr;
  uint4* d_uq = nullptr;
  int *d_key = nullptr, *d_scnt = nullptr, *d_sstart = nullptr, *d_scur = nullptr, *d_order = nullptr;
  Tan t{};
  unsigned* d_bar = nullptr;       // one word: XCC census of the persistent plan
  // persistent launch (planned by sw_set_tuning, allocated on first use)
  unsigned* d_pctl = nullptr;      // [kCtlWords] control words
  int* d_gtab = nullptr;           // replica groups (PArgs::gtab)
  size_t gtab_ints = 0;
  unsigned xmask = 0;              // XCC ids of the device (0: not taken yet)
  int pg_ng = 1;                   // groups of the plan (1: grid-wide barriers)
  int last_groups = 0;             // groups the last persistent call ran with
  // captured persistent call (persistent and graph_steps > 0)
  hipGraph_t pgraph = nullptr;
  hipGraphExec_t pgexec = nullptr;
  std::vector<unsigned char> pgkey;
  double* pring = nullptr;         // its thermo rows, copied out after each replay
  size_t pring_rows = 0;
  unsigned long long* d_audit = nullptr;   // [2] pairs within the cut-off audited, pairs missing from rows
  // captured block of steps (graph_steps > 0)
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<unsigned char> gkey;
  double* ring = nullptr;          // thermo rows of one captured block
  size_t ring_rows = 0;
  int alloc_gen = 0;               // bumped whenever capacity buffers move
  int last_grid = 0;               // blocks of the last persistent launch
  bool have_order = false;
  long long steps = 0;
  int last_hip = 0;
  std::unordered_map<void*, size_t> sizes;   // live device allocations
  std::vector<void*> allocs;       // everything freed by free_all
  std::vector<void*> grow_allocs;  // capacity-dependent buffers
  // adjoint work buffers (checkpoints, frame stores, adjoint vectors), kept
  // between calls and grown on demand; slot k is the k-th buffer a call asks for
  std::vector<void*> adj_buf;
  std::vector<size_t> adj_bytes;
  // captured adjoint core (graph_steps > 0), keyed by everything it reads
  hipGraph_t adj_graph = nullptr;
  hipGraphExec_t adj_gexec = nullptr;
  std::vector<unsigned char> adj_gkey;
  // observables (allocated on first use)
  double* obs_edges = nullptr;     // bin edges of the last histogram call
  unsigned long long* obs_flags = nullptr;   // [0] centres short of neighbours, [1] candidate overflow
  double* msd_last = nullptr;      // [N][3] caller order: positions at the last sample
  double* msd_acc = nullptr;       // [N][3] unwrapped displacement since the reference
  bool msd_ready = false;
  // isobaric dynamics (allocated on first use)
  swk::NptState* d_npt = nullptr;  // [2][R] double-buffered extended state
  swk::NptConst* d_nptc = nullptr; // [R]
  float2* d_kick = nullptr;        // [R] isobaric kick coefficients (Dev::npt_kick)
  std::vector<swk::NptState> npt;  // host copy between calls
  bool npt_ready = false;
  // captured block of isobaric steps (graph_steps > 0; shares cap_stream)
  hipGraph_t npt_graph = nullptr;
  hipGraphExec_t npt_gexec = nullptr;
  std::vector<unsigned char> npt_gkey;
  double* npt_ring = nullptr;      // records of one captured block
  size_t npt_ring_rows = 0;
};


namespace swh {
using namespace swk;

// Every device buffer of a context, in one place: `alloc(void** p, size_t
// bytes)` supplies the memory (hipMalloc in sw_create, a static scratch
// array in the allocation-free entry point).  place_buffers places the
// fixed-size ones, place_capacity_buffers the ones sized by the row and
// cell capacities (and records those capacities in the device view).
template <class A>
hipError_t place_buffers(sw_ctx* c, A&& alloc) {
  const size_t np = (size_t)c->npad;
  hipError_t e = hipSuccess;
  auto put = [&](auto*& ptr, size_t n) {
    if (e == hipSuccess) e = alloc((void**)&ptr, std::max<size_t>(n, 1) * sizeof(*ptr));
  };
  put(c->d.u[0], np); put(c->d.u[1], np); put(c->d.v, np); put(c->d.f, np); put(c->d.uref, np);
  put(c->d.ids, np); put(c->d.nn, np); put(c->d.nact, np); put(c->d.mom, 3 * np);
  put(c->d.gcnt[0], (size_t)c->ctot); put(c->d.gcnt[1], (size_t)c->ctot);
  put(c->d.partial, (np / kMinAPB + 1) * kNQ);   // one slot per block and quantity
  put(c->d.thermo_cur, (size_t)c->R * kNQ);
  put(c->d.arrive, (size_t)c->R);
  put(c->d.dflag, 2 * (size_t)c->R);
  put(c->d.flags, F_NFLAGS);
  put(c->d_bar, 1);
  put(c->d_audit, 2);
  put(c->d_reps, (size_t)c->R);
  put(c->d_tile_rep, c->tile_rep.size());
  put(c->d_uoff, (size_t)c->R + 1);
  put(c->d_cell_rank, (size_t)c->ctot);
  put(c->d_T0, (size_t)c->R);
  put(c->d.lref, (size_t)c->R);
  put(c->d_kick, (size_t)c->R);
  put(c->d_uq, (size_t)c->N); put(c->d_key, (size_t)c->N); put(c->d_order, (size_t)c->N);
  put(c->d_scnt, (size_t)c->ctot); put(c->d_sstart, (size_t)c->ctot); put(c->d_scur, (size_t)c->ctot);
  put(c->t.w, np); put(c->t.mdot, 3 * np); put(c->t.fdot, np); put(c->t.f3, np); put(c->t.gw, np);
  put(c->t.tpartial, (np / kMinAPB + 1) * kTQ);
  put(c->t.tsum, (size_t)c->R * kTQ);
  if (e != hipSuccess) return e;
  c->d.reps = c->d_reps;
  c->d.tile_rep = c->d_tile_rep;
  c->d.T0 = c->d_T0;
  c->d.npt_kick = c->d_kick;
  c->d.npad = c->npad;
  c->d.ctot = c->ctot;
  c->d.R = c->R;
  c->d.max_rep_pad = 0;
  for (const RepInfo& R : c->reps) c->d.max_rep_pad = std::max(c->d.max_rep_pad, R.ipad_end - R.ioff);
  return hipSuccess;
}

template <class A>
hipError_t place_capacity_buffers(sw_ctx* c, A&& alloc) {
  hipError_t e;
  if ((e = alloc((void**)&c->d.nl, sizeof(int) * (size_t)c->npad * c->cap)) != hipSuccess) return e;
  if ((e = alloc((void**)&c->d.act, sizeof(int) * (size_t)c->npad * c->cap)) != hipSuccess) return e;
  for (int k = 0; k < 2; ++k)
    if ((e = alloc((void**)&c->d.gmem[k], sizeof(uint4) * std::max<size_t>((size_t)c->ctot * c->cc, 1))) != hipSuccess)
      return e;
  c->d.cap = c->cap;
  c->d.cc = c->cc;
  return hipSuccess;
}

int setup_layout(sw_ctx* c, int n_replicas, const long long* h_offsets, const double* h_box, double cutoff,
                 double skin, int nbr_capacity);
int fail_hip(sw_ctx* c, hipError_t e);
int lpa_for(const sw_ctx* c);
int make_phys(const sw_ctx* c, const sw_params* P, double mass, double dt, Phys* o);
hipError_t reset_flags(sw_ctx* c, hipStream_t s);
struct Flags { int nbr_over, nbr_need, cell_over, overlap, abort, box, pgroups; };
hipError_t read_flags(sw_ctx* c, hipStream_t s, Flags* f);
int grow(sw_ctx* c, const Flags& f);
hipError_t sort_in(sw_ctx* c, const float* x, const float* v, hipStream_t s);
bool valid_ptr(const void* p);
int regrid(sw_ctx* c, double margin);
hipError_t dalloc_raw(sw_ctx* c, void** p, size_t bytes, std::vector<void*>& list);
size_t device_bytes(const sw_ctx* c);
}  // namespace swh
