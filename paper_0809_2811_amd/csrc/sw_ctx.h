// Host-side context of libsw, shared by sw_api.hip and sw_tangent.hip.
#pragma once
#include "sw.h"
#include "sw_internal.h"

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
  unsigned* d_bar = nullptr;       // grid barrier counter of the persistent launch
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
int fail_hip(sw_ctx* c, hipError_t e);
int lpa_for(const sw_ctx* c);
int make_phys(const sw_ctx* c, const sw_params* P, double mass, double dt, Phys* o);
hipError_t reset_flags(sw_ctx* c, hipStream_t s);
struct Flags { int nbr_over, nbr_need, cell_over, overlap, abort, box; };
hipError_t read_flags(sw_ctx* c, hipStream_t s, Flags* f);
int grow(sw_ctx* c, const Flags& f);
hipError_t sort_in(sw_ctx* c, const float* x, const float* v, hipStream_t s);
bool valid_ptr(const void* p);
int regrid(sw_ctx* c, double margin);
hipError_t dalloc_raw(sw_ctx* c, void** p, size_t bytes, std::vector<void*>& list);
size_t device_bytes(const sw_ctx* c);
}  // namespace swh
