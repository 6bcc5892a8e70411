// Host side of libsw: context management, argument checks and the C ABI
// declared in include/sw.h.  Every step of the computation runs in the HIP
// kernels of sw_kernels.hip (and sw_tangent.hip); this file only lays out
// memory, checks arguments and enqueues launches.

#include "sw.h"
#include "sw_ctx.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

using namespace swk;

namespace swh {

constexpr int kMaxCap = 512;
constexpr double kLog2e = 1.4426950408889634;

unsigned part1by2(unsigned x) {
  x &= 0x3ffu;
  x = (x | (x << 16)) & 0x030000ffu;
  x = (x | (x << 8)) & 0x0300f00fu;
  x = (x | (x << 4)) & 0x030c30c3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}

int fail_hip(sw_ctx* c, hipError_t e) {
  if (c) c->last_hip = (int)e;
  return SW_EHIP;
}

hipError_t dalloc_raw(sw_ctx* c, void** p, size_t bytes, std::vector<void*>& list) {
  *p = nullptr;
  if (bytes == 0) bytes = 1;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) return e;
  list.push_back(*p);
  c->sizes[*p] = bytes;
  return hipSuccess;
}

template <class T>
hipError_t dalloc(sw_ctx* c, T** p, size_t n, std::vector<void*>& list) {
  return dalloc_raw(c, (void**)p, std::max<size_t>(n, 1) * sizeof(T), list);
}

void free_list(sw_ctx* c, std::vector<void*>& list) {
  for (void* p : list) {
    (void)hipFree(p);
    c->sizes.erase(p);
  }
  list.clear();
}

// Frees one allocation of the context's main list.
void dfree(sw_ctx* c, void* p) {
  if (!p) return;
  (void)hipFree(p);
  c->sizes.erase(p);
  auto& L = c->allocs;
  L.erase(std::remove(L.begin(), L.end(), p), L.end());
}

size_t device_bytes(const sw_ctx* c) {
  size_t b = 0;
  for (const auto& kv : c->sizes) b += kv.second;
  return b;
}

// Morton rank of every cell of replica R (cells numbered from coff) into rank.
void cell_ranks(const RepInfo& R, int coff, std::vector<int>& rank) {
  std::vector<std::pair<unsigned, int>> codes(R.ncell);
  for (int x = 0; x < R.nc[0]; ++x)
    for (int y = 0; y < R.nc[1]; ++y)
      for (int z = 0; z < R.nc[2]; ++z) {
        const int local = (x * R.nc[1] + y) * R.nc[2] + z;
        codes[local] = {(part1by2(x) << 2) | (part1by2(y) << 1) | part1by2(z), local};
      }
  std::sort(codes.begin(), codes.end());
  rank.resize(coff + R.ncell);
  for (int k = 0; k < R.ncell; ++k) rank[coff + codes[k].second] = coff + k;
}

int lpa_for(const sw_ctx* c) {
  int lpa = c->tune.lanes_per_atom;
  // the rebuild's LDS staging grows with atoms per block and row capacity;
  // keep it within 64 KiB per block
  while (lpa < kMaxLPA && moments_lds_bytes(kBlock / lpa, c->cap) > 65536) lpa *= 2;
  return lpa;
}

// Buffers whose size depends on the row and cell capacities.
hipError_t alloc_capacity(sw_ctx* c) {
  free_list(c, c->grow_allocs);
  hipError_t e = place_capacity_buffers(c, [c](void** p, size_t bytes) { return dalloc_raw(c, p, bytes, c->grow_allocs); });
  if (e != hipSuccess) return e;
  ++c->alloc_gen;
  return hipSuccess;
}

hipError_t alloc_all(sw_ctx* c) {
  hipError_t e;
  if ((e = place_buffers(c, [c](void** p, size_t bytes) { return dalloc_raw(c, p, bytes, c->allocs); })) != hipSuccess)
    return e;
  if ((e = alloc_capacity(c)) != hipSuccess) return e;
  if ((e = hipMemcpy(c->d_reps, c->reps.data(), sizeof(RepInfo) * c->R, hipMemcpyHostToDevice)) != hipSuccess) return e;
  if ((e = hipMemcpy(c->d_tile_rep, c->tile_rep.data(), sizeof(int) * c->tile_rep.size(), hipMemcpyHostToDevice)) != hipSuccess) return e;
  if ((e = hipMemcpy(c->d_uoff, c->uoff.data(), sizeof(long long) * (c->R + 1), hipMemcpyHostToDevice)) != hipSuccess) return e;
  if ((e = hipMemcpy(c->d_cell_rank, c->cell_rank.data(), sizeof(int) * c->ctot, hipMemcpyHostToDevice)) != hipSuccess) return e;
  if ((e = hipMemset(c->d.arrive, 0, sizeof(int) * c->R)) != hipSuccess) return e;
  if ((e = hipMemset(c->d.flags, 0, sizeof(int) * F_NFLAGS)) != hipSuccess) return e;
  if ((e = hipMemset(c->d_audit, 0, sizeof(unsigned long long) * 2)) != hipSuccess) return e;
  if ((e = hipMemset(c->d.dflag, 0, sizeof(int) * 2 * c->R)) != hipSuccess) return e;
  if ((e = hipMemset(c->d.thermo_cur, 0, sizeof(double) * kNQ * c->R)) != hipSuccess) return e;
  return hipSuccess;
}

// Replica layout of a context (no device work): boxes, binning grids,
// Morton ranks of the cells, 64-atom tiles, padded atom ranges, initial row
// and cell capacities.  Returns SW_OK, SW_EINVAL or SW_EBOX_TOO_SMALL.
int setup_layout(sw_ctx* c, int n_replicas, const long long* h_offsets, const double* h_box, double cutoff,
                 double skin, int nbr_capacity) {
  if (n_replicas <= 0 || !h_offsets || !h_box || !(cutoff > 0.0) || !(skin >= 0.0) || nbr_capacity <= 0 ||
      nbr_capacity > kMaxCap || !std::isfinite(cutoff) || !std::isfinite(skin))
    return SW_EINVAL;
  if (h_offsets[0] != 0) return SW_EINVAL;
  for (int r = 0; r < n_replicas; ++r) {
    if (h_offsets[r + 1] - h_offsets[r] < 2) return SW_EINVAL;
    for (int k = 0; k < 3; ++k)
      if (!(h_box[3 * r + k] > 0.0) || !std::isfinite(h_box[3 * r + k])) return SW_EINVAL;
  }
  if (h_offsets[n_replicas] >= (1LL << 30)) return SW_EINVAL;
  c->R = n_replicas;
  c->N = h_offsets[n_replicas];
  c->uoff.assign(h_offsets, h_offsets + n_replicas + 1);
  c->box.assign(h_box, h_box + 3 * n_replicas);
  c->cutoff = cutoff;
  c->skin = skin;
  c->cap = (nbr_capacity + 3) & ~3;
  const double rl = cutoff + skin;
  int ioff = 0, coff = 0;
  c->reps.clear();
  c->tile_rep.clear();
  c->cell_rank.clear();
  for (int r = 0; r < n_replicas; ++r) {
    RepInfo R{};
    const int n = (int)(h_offsets[r + 1] - h_offsets[r]);
    for (int k = 0; k < 3; ++k) {
      const double L = h_box[3 * r + k];
      R.L[k] = L;
      R.scale[k] = (float)(L / kTwo32);
      R.inv_scale[k] = (float)(kTwo32 / L);
      const int nc = (int)std::floor(L / rl);
      if (nc < 3) return SW_EBOX_TOO_SMALL;
      R.nc[k] = std::min(nc, 1024);
    }
    R.ncell = R.nc[0] * R.nc[1] * R.nc[2];
    R.cell_off = coff;
    R.ioff = ioff;
    R.n = n;
    R.iend = ioff + n;
    R.ipad_end = ioff + ((n + kTile - 1) / kTile) * kTile;
    R.uoff = h_offsets[r];
    R.ndof_kb = (3.0 * n - 3.0) * kBoltz;
    cell_ranks(R, coff, c->cell_rank);
    for (int t = ioff / kTile; t < R.ipad_end / kTile; ++t) c->tile_rep.push_back(r);
    ioff = R.ipad_end;
    coff += R.ncell;
    c->reps.push_back(R);
  }
  c->npad = ioff;
  c->ctot = coff;
  // binning cells hold ~ n * rl^3 atoms on average; start at 4x that, min 32
  double mean = 0.0;
  for (const auto& R : c->reps) mean = std::max(mean, (double)R.n / R.ncell);
  c->cc = std::max(32, (int)std::ceil(4.0 * mean / 8.0) * 8);
  return SW_OK;
}

int make_phys(const sw_ctx* c, const sw_params* P, double mass, double dt, Phys* o) {
  if (!P) return SW_EINVAL;
  if (P->p != 4.0 || P->q != 0.0) return SW_EUNSUPPORTED;
  const double rc = P->a * P->sigma;
  if (!(rc > 0.0) || !(P->sigma > 0.0) || !(P->epsilon > 0.0) || !std::isfinite(P->lambda) ||
      !std::isfinite(P->gamma) || !std::isfinite(P->cos_theta0))
    return SW_EINVAL;
  if (rc > c->cutoff * (1.0 + 1e-12)) return SW_EINVAL;
  const double rl = c->cutoff + c->skin;
  o->rc = (float)rc;
  // Pairs are accepted on r^2 < rc2, but the radial factors then take
  // r = r^2 rsq(r^2) with the hardware reciprocal square root (within 1 ulp):
  // for an r^2 just below rc^2 that r can round to rc or past it, and
  // exp(gamma sigma / (r - rc)) becomes exp(+inf).  rc2 sits 2^-20 (relative)
  // below rc^2 so that every accepted pair has r < rc in float; over that
  // sliver (about 2e-6 A) both exponential factors are exactly zero in float.
  o->rc2 = (float)((double)o->rc * (double)o->rc * (1.0 - 0x1p-20));
  o->rl2 = (float)(rl * rl);
  o->half_skin = (float)(0.5 * (rl - rc) - 1e-4);
  o->sig = (float)P->sigma;
  o->sig_l2e = (float)(P->sigma * kLog2e);
  o->gsig = (float)(P->gamma * P->sigma);
  o->gsig_l2e = (float)(P->gamma * P->sigma * kLog2e);
  o->Aeps = (float)(P->A * P->epsilon);
  o->B = (float)P->B;
  o->lameps = (float)(P->lambda * P->epsilon);
  o->c0 = (float)P->cos_theta0;
  o->qc = (float)((1.0 - P->cos_theta0) * (1.0 - P->cos_theta0));
  const double m = mass > 0.0 ? mass : 1.0;
  o->hdt_cm = (float)(0.5 * dt * kAcc / m);
  o->dt = (float)dt;
  o->half_m_acc = (float)(0.5 * m / kAcc);
  o->m_acc = (float)(m / kAcc);
  o->dt_d = dt;
  o->tau_d = 1.0;
  o->thermostat = 0;
  o->term2 = 1.f;
  o->term3 = 1.f;
  return SW_OK;
}

hipError_t reset_flags(sw_ctx* c, hipStream_t s) {
  // keep the cumulative rebuild counter (slot F_REBUILDS)
  hipError_t e = launch_fill_i32(c->d.flags, 0, F_REBUILDS, s);
  if (e != hipSuccess) return e;
  return launch_fill_i32(c->d.dflag, 0, 2 * c->R, s);
}

hipError_t read_flags(sw_ctx* c, hipStream_t s, Flags* f) {
  int h[F_NFLAGS];
  hipError_t e = hipMemcpyAsync(h, c->d.flags, sizeof h, hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  f->nbr_over = h[F_NBR_OVER];
  f->nbr_need = h[F_NBR_NEED];
  f->cell_over = h[F_CELL_OVER];
  f->overlap = h[F_OVERLAP];
  f->abort = h[F_ABORT];
  f->box = h[F_BOX];
  f->pgroups = h[F_PGROUPS];
  return hipSuccess;
}

// Grows the capacities named by the flags.  Returns SW_OK if something grew.
int grow(sw_ctx* c, const Flags& f) {
  bool grew = false;
  if (f.nbr_over) {
    int need = std::max(f.nbr_need + f.nbr_need / 4 + 4, c->cap + 8);
    need = (need + 3) & ~3;
    if (c->cap >= kMaxCap) return SW_ENBR_OVERFLOW;
    c->cap = std::min(need, kMaxCap);
    grew = true;
  }
  if (f.cell_over) {
    if (c->cc >= 4096) return SW_ECELL_OVERFLOW;
    c->cc *= 2;
    grew = true;
  }
  if (!grew) return SW_EINVAL;
  hipError_t e = alloc_capacity(c);
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? SW_ENOMEM : fail_hip(c, e);
  c->have_order = false;
  return SW_OK;
}

// Recomputes every replica's binning grid from its current box so that a
// cell edge is at least (cutoff + skin)(1 + margin), and reallocates the
// grid-sized buffers if the grid changed.
int regrid(sw_ctx* c, double margin) {
  const double rl = c->cutoff + c->skin;
  bool same = true;
  std::vector<RepInfo> reps = c->reps;
  for (int r = 0; r < c->R; ++r)
    for (int k = 0; k < 3; ++k) {
      const int nc = std::min((int)std::floor(c->box[3 * r + k] / (rl * (1.0 + margin))), 1024);
      if (nc < 3) return SW_EBOX_TOO_SMALL;
      same = same && nc == reps[r].nc[k];
      reps[r].nc[k] = nc;
    }
  if (same) return SW_OK;
  std::vector<int> rank;
  int coff = 0;
  for (auto& R : reps) {
    R.ncell = R.nc[0] * R.nc[1] * R.nc[2];
    R.cell_off = coff;
    cell_ranks(R, coff, rank);
    coff += R.ncell;
  }
  c->reps = reps;
  c->cell_rank = rank;
  c->ctot = coff;
  hipError_t e;
  for (int** p : {&c->d.gcnt[0], &c->d.gcnt[1], &c->d_cell_rank, &c->d_scnt, &c->d_sstart, &c->d_scur}) {
    dfree(c, *p);
    if ((e = dalloc(c, p, (size_t)c->ctot, c->allocs)) != hipSuccess)
      return e == hipErrorOutOfMemory ? SW_ENOMEM : fail_hip(c, e);
  }
  if ((e = alloc_capacity(c)) != hipSuccess) return e == hipErrorOutOfMemory ? SW_ENOMEM : fail_hip(c, e);
  c->d.ctot = c->ctot;
  if ((e = hipMemcpy(c->d_reps, c->reps.data(), sizeof(RepInfo) * c->R, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(c->d_cell_rank, c->cell_rank.data(), sizeof(int) * c->ctot, hipMemcpyHostToDevice)) !=
          hipSuccess)
    return fail_hip(c, e);
  c->have_order = false;
  return SW_OK;
}

// Sort the caller's atoms along the Morton curve of the binning cells, load
// them (and velocities if given) into internal order, bin into grid 0.
hipError_t sort_in(sw_ctx* c, const float* x, const float* v, hipStream_t s) {
  hipError_t e = launch_sort(c->d, (const float4*)x, (const float4*)v, c->N, c->d_uoff, c->R, c->d_cell_rank,
                             c->d_uq, c->d_key, c->d_scnt, c->d_sstart, c->d_scur, c->d_order, s);
  if (e != hipSuccess) return e;
  if ((e = launch_fill_i32(c->d.gcnt[0], 0, c->ctot, s)) != hipSuccess) return e;
  if ((e = launch_bin(c->d, 0, 0, 0.f, 0.f, s)) != hipSuccess) return e;
  c->have_order = true;
  return hipSuccess;
}

bool valid_ptr(const void* p) { return p != nullptr; }

// Enqueues step t of the per-phase path.  row: thermo destination or null.
hipError_t enqueue_step(sw_ctx* c, const Phys& ph, int lpa, int t, int nsteps, int thermostat, bool rec,
                        double* row, hipStream_t s, const KTimer& tm_m, const KTimer& tm_f) {
  const int par = t & 1;
  const int force_rb = c->tune.rebuild_every > 0 && (t % c->tune.rebuild_every == 0);
  hipError_t e;
  if ((e = launch_moments(c->d, ph, lpa, par, force_rb, rec, s, tm_m)) != hipSuccess) return e;
  if (c->tune.audit_every > 0 && t % c->tune.audit_every == 0 &&
      (e = launch_audit(c->d, ph, par, c->d_audit, s)) != hipSuccess)
    return e;
  if (thermostat == SW_NVE) {
    const int mode = t == nsteps ? MODE_NVE_LAST : MODE_NVE;
    if ((e = launch_forces(c->d, ph, lpa, mode, rec, par, row, s, tm_f)) != hipSuccess) return e;
  } else {
    if ((e = launch_forces(c->d, ph, lpa, MODE_KICK, rec, par, row, s, tm_f)) != hipSuccess) return e;
    if ((e = launch_thermostat(c->d, ph, lpa, par, t == nsteps, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

long long lcm_ll(long long a, long long b) {
  long long x = a, y = b;
  while (y) { long long r = x % y; x = y; y = r; }
  return a / x * b;
}

// Captures steps base+1 .. base+K (base a multiple of the pattern period) of
// the per-phase path into a graph, unless the cached one matches.
hipError_t ensure_graph(sw_ctx* c, const Phys& ph, int lpa, int K, int thermostat, int every) {
  std::vector<unsigned char> key(sizeof(Phys) + 8 * sizeof(int));
  int meta[8] = {K, lpa, thermostat, every, c->tune.rebuild_every, c->alloc_gen, c->d.sync_rb, c->tune.audit_every};
  std::memcpy(key.data(), &ph, sizeof(Phys));
  std::memcpy(key.data() + sizeof(Phys), meta, sizeof meta);
  if (c->gexec && key == c->gkey) return hipSuccess;
  hipError_t e;
  if (c->gexec) { (void)hipGraphExecDestroy(c->gexec); c->gexec = nullptr; }
  if (c->graph) { (void)hipGraphDestroy(c->graph); c->graph = nullptr; }
  if (!c->cap_stream && (e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking)) != hipSuccess) return e;
  const size_t rows = every > 0 ? (size_t)(K / every) : 0;
  if (rows > c->ring_rows) {
    if (c->ring) (void)hipFree(c->ring);
    c->ring = nullptr;
    c->ring_rows = 0;
    if ((e = hipMalloc((void**)&c->ring, rows * c->R * kNQ * sizeof(double))) != hipSuccess) return e;
    c->ring_rows = rows;
  }
  if ((e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
  hipError_t le = hipSuccess;
  for (int l = 1; l <= K && le == hipSuccess; ++l) {
    const bool rec = every > 0 && l % every == 0;
    double* row = rec ? c->ring + (size_t)(l / every - 1) * c->R * kNQ : nullptr;
    // local step l stands for step base + l; the last step of a call is never captured
    le = enqueue_step(c, ph, lpa, l, K + 1, thermostat, rec, row, c->cap_stream, KTimer(), KTimer());
  }
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(c->cap_stream, &g);
  if (le != hipSuccess) { if (g) (void)hipGraphDestroy(g); return le; }
  if (e != hipSuccess) return e;
  c->graph = g;
  if ((e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0)) != hipSuccess) return e;
  c->gkey = key;
  return hipSuccess;
}

// The persistent launches of one sw_step call (steps 1..nsteps), in
// launches of at most kPersistSteps steps; thermo rows go to `rows`.
hipError_t enqueue_persistent(sw_ctx* c, const Phys& ph, int lpa, int nsteps, int every, double* rows,
                              hipStream_t s) {
  hipError_t e = hipSuccess;
  for (int t0 = 1; t0 <= nsteps && e == hipSuccess; t0 += kPersistSteps) {
    const int t1 = std::min(nsteps, t0 + kPersistSteps - 1);
    PArgs pa{t0, t1, nsteps, rows ? every : 0, c->tune.rebuild_every, rows, c->d_pctl, c->d.flags + F_ABORT,
             c->d.sync_rb, c->pg_ng, c->xmask, c->d_gtab};
    e = launch_persistent(c->d, ph, lpa, pa, c->tune.persistent > 1 ? c->tune.persistent : 0, s, &c->last_grid);
  }
  return e;
}

// A captured copy of a call's persistent launches (the control-word fills
// and cooperative launches of enqueue_persistent), keyed by everything
// they read; thermo rows land in pring.
hipError_t ensure_pgraph(sw_ctx* c, const Phys& ph, int lpa, int nsteps, int every) {
  std::vector<unsigned char> key(sizeof(Phys) + 12 * sizeof(int));
  const unsigned long long tab = (unsigned long long)(size_t)c->d_gtab;
  int meta[12] = {nsteps, lpa, every, c->tune.rebuild_every, c->alloc_gen, c->d.sync_rb, c->pg_ng, (int)c->xmask,
                  c->tune.persistent, (int)(tab & 0xffffffffu), (int)(tab >> 32), c->R};
  std::memcpy(key.data(), &ph, sizeof(Phys));
  std::memcpy(key.data() + sizeof(Phys), meta, sizeof meta);
  if (c->pgexec && key == c->pgkey) return hipSuccess;
  hipError_t e;
  if (c->pgexec) { (void)hipGraphExecDestroy(c->pgexec); c->pgexec = nullptr; }
  if (c->pgraph) { (void)hipGraphDestroy(c->pgraph); c->pgraph = nullptr; }
  c->pgkey.clear();
  if (!c->cap_stream && (e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking)) != hipSuccess) return e;
  const size_t rows = every > 0 ? (size_t)(nsteps / every) : 0;
  if (rows > c->pring_rows) {
    if (c->pring) (void)hipFree(c->pring);
    c->pring = nullptr;
    c->pring_rows = 0;
    if ((e = hipMalloc((void**)&c->pring, rows * c->R * kNQ * sizeof(double))) != hipSuccess) return e;
    c->pring_rows = rows;
  }
  if ((e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
  const hipError_t le = enqueue_persistent(c, ph, lpa, nsteps, every, rows ? c->pring : nullptr, c->cap_stream);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(c->cap_stream, &g);
  if (le != hipSuccess) { if (g) (void)hipGraphDestroy(g); return le; }
  if (e != hipSuccess) return e;
  c->pgraph = g;
  if ((e = hipGraphInstantiate(&c->pgexec, g, nullptr, nullptr, 0)) != hipSuccess) return e;
  c->pgkey = key;
  return hipSuccess;
}

}  // namespace swh

using namespace swh;

extern "C" {

void sw_params_mw(sw_params* out) {
  if (!out) return;
  out->lambda = 23.15;
  out->epsilon = 6.189;
  out->sigma = 2.3925;
  out->A = 7.049556277;
  out->B = 0.6022245584;
  out->p = 4.0;
  out->q = 0.0;
  out->gamma = 1.2;
  out->a = 1.8;
  out->cos_theta0 = -1.0 / 3.0;
}

const char* sw_status_string(int s) {
  switch (s) {
    case SW_OK: return "ok";
    case SW_EINVAL: return "invalid argument";
    case SW_EBOX_TOO_SMALL: return "box edge shorter than three cells of cutoff + skin";
    case SW_ENBR_OVERFLOW: return "neighbour row capacity exceeded";
    case SW_ECELL_OVERFLOW: return "binning cell capacity exceeded";
    case SW_EOVERLAP: return "atoms overlap (< 0.5 A), non-finite values, or a step longer than a quarter box";
    case SW_EHIP: return "HIP runtime error";
    case SW_ENOMEM: return "device memory exhausted";
    case SW_EUNSUPPORTED: return "unsupported parameter or option";
    case SW_ESTATE: return "context has no neighbour rows yet";
    case SW_ETIMEOUT: return "a grid barrier of the persistent launch waited too long";
    case SW_ESCRATCH: return "input too large for the allocation-free entry point's static scratch";
  }
  return "unknown status";
}

int sw_last_hip_error(const sw_ctx* ctx) { return ctx ? ctx->last_hip : 0; }

int sw_create(sw_ctx** out, int n_replicas, const long long* h_offsets, const double* h_box, double cutoff,
              double skin, int nbr_capacity) {
  if (!out) return SW_EINVAL;
  *out = nullptr;
  sw_ctx* c = new (std::nothrow) sw_ctx;
  if (!c) return SW_ENOMEM;
  const int st = setup_layout(c, n_replicas, h_offsets, h_box, cutoff, skin, nbr_capacity);
  if (st != SW_OK) {
    delete c;
    return st;
  }
  hipError_t e = alloc_all(c);
  if (e != hipSuccess) {
    free_list(c, c->grow_allocs);
    free_list(c, c->allocs);
    delete c;
    return e == hipErrorOutOfMemory ? SW_ENOMEM : SW_EHIP;
  }
  *out = c;
  return SW_OK;
}

void sw_destroy(sw_ctx* ctx) {
  if (!ctx) return;
  (void)hipDeviceSynchronize();
  for (hipEvent_t e : ctx->tev) (void)hipEventDestroy(e);
  if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->ring) (void)hipFree(ctx->ring);
  if (ctx->npt_gexec) (void)hipGraphExecDestroy(ctx->npt_gexec);
  if (ctx->npt_graph) (void)hipGraphDestroy(ctx->npt_graph);
  if (ctx->npt_ring) (void)hipFree(ctx->npt_ring);
  if (ctx->adj_gexec) (void)hipGraphExecDestroy(ctx->adj_gexec);
  if (ctx->adj_graph) (void)hipGraphDestroy(ctx->adj_graph);
  for (void* p : ctx->adj_buf) (void)hipFree(p);
  if (ctx->pgexec) (void)hipGraphExecDestroy(ctx->pgexec);
  if (ctx->pgraph) (void)hipGraphDestroy(ctx->pgraph);
  if (ctx->pring) (void)hipFree(ctx->pring);
  if (ctx->d_pctl) (void)hipFree(ctx->d_pctl);
  if (ctx->d_gtab) (void)hipFree(ctx->d_gtab);
  free_list(ctx, ctx->grow_allocs);
  free_list(ctx, ctx->allocs);
  delete ctx;
}

// Plan of the persistent launch (k_persistent): its control words, the XCC
// ids of the device, and the replica groups.  Replicas are dealt to the
// XCCs largest first, each to the least loaded group; the group form is
// kept only if no group holds more than 1.25 times the mean load (a
// context of fewer replicas than XCCs, or one dominated by a replica, runs
// the grid form).  The plan depends on the replica sizes alone.
static int plan_persistent(sw_ctx* c) {
  hipError_t e;
  if (!c->d_pctl && (e = hipMalloc((void**)&c->d_pctl, sizeof(unsigned) * kCtlWords)) != hipSuccess)
    return e == hipErrorOutOfMemory ? SW_ENOMEM : fail_hip(c, e);
  if (c->xmask == 0 && (e = xcc_census(c->d_bar, &c->xmask, nullptr)) != hipSuccess) return fail_hip(c, e);
  c->pg_ng = 1;
  const int nx = __builtin_popcount(c->xmask);
  if (nx < 2 || c->R < nx) return SW_OK;
  std::vector<long long> load(nx, 0);
  std::vector<int> order(c->R), grp(c->R);
  for (int r = 0; r < c->R; ++r) order[r] = r;
  auto waves = [&](int r) { return (long long)(c->reps[r].ipad_end - c->reps[r].ioff) / kTile; };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return waves(x) > waves(y); });
  long long total = 0;
  for (int r : order) {
    const int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    grp[r] = g;
    load[g] += waves(r);
    total += waves(r);
  }
  if ((double)*std::max_element(load.begin(), load.end()) * nx > 1.25 * (double)total) return SW_OK;
  std::vector<int> tab(2 * (nx + 1) + c->R);
  int* woff = tab.data();
  int* roff = woff + nx + 1;
  int* reps = roff + nx + 1;
  int nr = 0;
  for (int g = 0; g < nx; ++g) {
    woff[g + 1] = woff[g] + (int)load[g];
    roff[g] = nr;
    for (int r = 0; r < c->R; ++r)
      if (grp[r] == g) reps[nr++] = r;
  }
  roff[nx] = nr;
  if (c->gtab_ints < tab.size()) {
    if (c->d_gtab) (void)hipFree(c->d_gtab);
    c->d_gtab = nullptr;
    c->gtab_ints = 0;
    if ((e = hipMalloc((void**)&c->d_gtab, sizeof(int) * tab.size())) != hipSuccess)
      return e == hipErrorOutOfMemory ? SW_ENOMEM : fail_hip(c, e);
    c->gtab_ints = tab.size();
  }
  if ((e = hipMemcpy(c->d_gtab, tab.data(), sizeof(int) * tab.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return fail_hip(c, e);
  c->pg_ng = nx;
  return SW_OK;
}

int sw_set_tuning(sw_ctx* ctx, const sw_tuning* t) {
  if (!ctx || !t) return SW_EINVAL;
  if (t->lanes_per_atom != 4 && t->lanes_per_atom != 8 && t->lanes_per_atom != 16 && t->lanes_per_atom != 32 &&
      t->lanes_per_atom != 64)
    return SW_EUNSUPPORTED;
  if (t->graph_steps < 0 || t->rebuild_every < 0 || t->timing < 0 || t->persistent < 0 || t->audit_every < 0)
    return SW_EINVAL;
  if (t->sync_rebuild != 0 && t->sync_rebuild != 1) return SW_EINVAL;
  if (t->persistent > 0) {
    const int st = plan_persistent(ctx);
    if (st != SW_OK) return st;
  }
  ctx->tune = *t;
  ctx->d.sync_rb = t->sync_rebuild;
  ctx->t_mom_ms = ctx->t_for_ms = 0.0;
  ctx->t_samples = 0;
  return SW_OK;
}

int sw_get_tuning(const sw_ctx* ctx, sw_tuning* t) {
  if (!ctx || !t) return SW_EINVAL;
  *t = ctx->tune;
  return SW_OK;
}

int sw_build_neighbors(sw_ctx* ctx, const float* x, void* stream) {
  if (!ctx || !valid_ptr(x)) return SW_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  sw_params P;
  sw_params_mw(&P);
  P.a = ctx->cutoff / P.sigma;  // rows only need the row radius; moments use the full cut-off
  Phys ph{};
  int st = make_phys(ctx, &P, 1.0, 1.0, &ph);
  if (st != SW_OK) return st;
  for (int attempt = 0; attempt < 6; ++attempt) {
    hipError_t e;
    if ((e = reset_flags(ctx, s)) != hipSuccess) return fail_hip(ctx, e);
    if ((e = sort_in(ctx, x, nullptr, s)) != hipSuccess) return fail_hip(ctx, e);
    if ((e = launch_moments(ctx->d, ph, lpa_for(ctx), 0, 1, 0, s)) != hipSuccess) return fail_hip(ctx, e);
    Flags f;
    if ((e = read_flags(ctx, s, &f)) != hipSuccess) return fail_hip(ctx, e);
    if (!f.nbr_over && !f.cell_over) return SW_OK;
    if ((st = grow(ctx, f)) != SW_OK) return st;
  }
  return SW_ENBR_OVERFLOW;
}

int sw_get_neighbors(sw_ctx* ctx, int* h_counts, int* h_rows, int max_per_row) {
  if (!ctx || !h_counts || !h_rows || max_per_row <= 0) return SW_EINVAL;
  if (!ctx->have_order) return SW_ESTATE;
  const size_t np = ctx->npad;
  std::vector<int> nn(np), ids(np), nl(np * ctx->cap);
  hipError_t e;
  if ((e = hipDeviceSynchronize()) != hipSuccess) return fail_hip(ctx, e);
  if ((e = hipMemcpy(nn.data(), ctx->d.nn, sizeof(int) * np, hipMemcpyDeviceToHost)) != hipSuccess) return fail_hip(ctx, e);
  if ((e = hipMemcpy(ids.data(), ctx->d.ids, sizeof(int) * np, hipMemcpyDeviceToHost)) != hipSuccess) return fail_hip(ctx, e);
  if ((e = hipMemcpy(nl.data(), ctx->d.nl, sizeof(int) * np * ctx->cap, hipMemcpyDeviceToHost)) != hipSuccess) return fail_hip(ctx, e);
  for (size_t i = 0; i < np; ++i) {
    const int k = ids[i];
    if (k < 0) continue;
    if (nn[i] > max_per_row) return SW_EINVAL;
    h_counts[k] = nn[i];
    int* row = h_rows + (size_t)k * max_per_row;
    for (int s = 0; s < nn[i]; ++s) row[s] = ids[nl[i * ctx->cap + s]];
    std::sort(row, row + nn[i]);
    for (int s = nn[i]; s < max_per_row; ++s) row[s] = -1;
  }
  return SW_OK;
}

int sw_forces(sw_ctx* ctx, const float* x, const sw_params* params, float* f, double* energy, double* virial,
              void* stream) {
  if (!ctx || !valid_ptr(x) || !valid_ptr(f)) return SW_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  Phys ph{};
  int st = make_phys(ctx, params, 1.0, 1.0, &ph);
  if (st != SW_OK) return st;
  for (int attempt = 0; attempt < 6; ++attempt) {
    hipError_t e;
    if ((e = reset_flags(ctx, s)) != hipSuccess) return fail_hip(ctx, e);
    int force_rebuild = 0;
    if (!ctx->have_order) {
      if ((e = sort_in(ctx, x, nullptr, s)) != hipSuccess) return fail_hip(ctx, e);
      force_rebuild = 1;
    } else {
      if ((e = launch_gather_ids(ctx->d, (const float4*)x, 0, s)) != hipSuccess) return fail_hip(ctx, e);
      if ((e = launch_fill_i32(ctx->d.gcnt[0], 0, ctx->ctot, s)) != hipSuccess) return fail_hip(ctx, e);
      if ((e = launch_bin(ctx->d, 0, 1, (float)(ctx->cutoff + ctx->skin), ph.rc, s)) != hipSuccess) return fail_hip(ctx, e);
    }
    const int lpa = lpa_for(ctx);
    if ((e = launch_moments(ctx->d, ph, lpa, 0, force_rebuild, 1, s)) != hipSuccess) return fail_hip(ctx, e);
    if ((e = launch_forces(ctx->d, ph, lpa, MODE_FORCES, 1, 0, nullptr, s)) != hipSuccess) return fail_hip(ctx, e);
    Flags fl;
    if ((e = read_flags(ctx, s, &fl)) != hipSuccess) return fail_hip(ctx, e);
    if (fl.nbr_over || fl.cell_over) {
      if ((st = grow(ctx, fl)) != SW_OK) return st;
      continue;
    }
    if ((e = launch_scatter_out(ctx->d, 0, nullptr, nullptr, (float4*)f, s)) != hipSuccess) return fail_hip(ctx, e);
    if ((energy || virial) && (e = launch_copy_thermo(ctx->d, energy, virial, s)) != hipSuccess)
      return fail_hip(ctx, e);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail_hip(ctx, e);
    return fl.overlap ? SW_EOVERLAP : SW_OK;
  }
  return SW_ENBR_OVERFLOW;
}

int sw_step(sw_ctx* ctx, float* x, float* v, float* f, const sw_params* params, double mass, double dt,
            int nsteps, int thermostat, const double* h_T0, double tau_fs, double* thermo, int thermo_every,
            void* stream) {
  if (!ctx || !valid_ptr(x) || !valid_ptr(v) || !valid_ptr(f)) return SW_EINVAL;
  if (!(mass > 0.0) || !(dt > 0.0) || nsteps < 0 || !std::isfinite(mass) || !std::isfinite(dt)) return SW_EINVAL;
  if (thermostat < SW_NVE || thermostat > SW_BERENDSEN) return SW_EINVAL;
  if (thermostat != SW_NVE && !h_T0) return SW_EINVAL;
  if (thermostat == SW_BERENDSEN && !(tau_fs > 0.0)) return SW_EINVAL;
  if (thermo && thermo_every <= 0) return SW_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  Phys ph{};
  int st = make_phys(ctx, params, mass, dt, &ph);
  if (st != SW_OK) return st;
  ph.thermostat = thermostat;
  ph.tau_d = thermostat == SW_BERENDSEN ? tau_fs : 1.0;
  hipError_t e;
  if (thermostat != SW_NVE) {
    for (int r = 0; r < ctx->R; ++r)
      if (!(h_T0[r] >= 0.0) || !std::isfinite(h_T0[r])) return SW_EINVAL;
    if ((e = hipMemcpyAsync(ctx->d_T0, h_T0, sizeof(double) * ctx->R, hipMemcpyHostToDevice, s)) != hipSuccess)
      return fail_hip(ctx, e);
  }
  const int lpa = lpa_for(ctx);
  const int period = ctx->tune.timing;
  const int max_samples = period > 0 ? std::min(256, nsteps / period) : 0;
  while ((int)ctx->tev.size() < 4 * max_samples) {
    hipEvent_t ev;
    if ((e = hipEventCreate(&ev)) != hipSuccess) return fail_hip(ctx, e);
    ctx->tev.push_back(ev);
  }
  for (int attempt = 0; attempt < 6; ++attempt) {
    int samples = 0;
    if ((e = reset_flags(ctx, s)) != hipSuccess) return fail_hip(ctx, e);
    if ((e = sort_in(ctx, x, v, s)) != hipSuccess) return fail_hip(ctx, e);
    if ((e = launch_moments(ctx->d, ph, lpa, 0, 1, 0, s)) != hipSuccess) return fail_hip(ctx, e);
    if (nsteps == 0) {
      if ((e = launch_forces(ctx->d, ph, lpa, MODE_FORCES, 1, 0, nullptr, s)) != hipSuccess) return fail_hip(ctx, e);
    } else {
      if ((e = launch_forces(ctx->d, ph, lpa, MODE_START, 0, 0, nullptr, s)) != hipSuccess) return fail_hip(ctx, e);
      const bool persistent = ctx->tune.persistent > 0;
      if (persistent && ctx->tune.graph_steps > 0) {
        // the call's persistent launches replayed from a captured graph
        const int every = thermo ? thermo_every : 0;
        if ((e = ensure_pgraph(ctx, ph, lpa, nsteps, every)) != hipSuccess) return fail_hip(ctx, e);
        if ((e = hipGraphLaunch(ctx->pgexec, s)) != hipSuccess) return fail_hip(ctx, e);
        if (every > 0 && nsteps / every > 0 &&
            (e = hipMemcpyAsync(thermo, ctx->pring, (size_t)(nsteps / every) * ctx->R * kNQ * sizeof(double),
                                hipMemcpyDeviceToDevice, s)) != hipSuccess)
          return fail_hip(ctx, e);
      } else if (persistent) {
        if ((e = enqueue_persistent(ctx, ph, lpa, nsteps, thermo ? thermo_every : 0, thermo, s)) != hipSuccess)
          return fail_hip(ctx, e);
      }
      int t_first = 1;
      if (!persistent && ctx->tune.graph_steps > 0 && nsteps > 1) {
        // replay a captured block of K steps over steps 1 .. nsteps-1 where
        // the block pattern (parity, thermo rows, forced rebuilds) repeats
        long long period = 2;
        const int every = thermo ? thermo_every : 0;
        if (every > 0) period = lcm_ll(period, every);
        if (ctx->tune.rebuild_every > 0) period = lcm_ll(period, ctx->tune.rebuild_every);
        if (ctx->tune.audit_every > 0) period = lcm_ll(period, ctx->tune.audit_every);
        const long long K = ((ctx->tune.graph_steps + period - 1) / period) * period;
        const long long nblk = (nsteps - 1) / K;
        if (nblk > 0 && K <= 1 << 20) {
          if ((e = ensure_graph(ctx, ph, lpa, (int)K, thermostat, every)) != hipSuccess) return fail_hip(ctx, e);
          for (long long b = 0; b < nblk; ++b) {
            if ((e = hipGraphLaunch(ctx->gexec, s)) != hipSuccess) return fail_hip(ctx, e);
            if (every > 0) {
              const size_t rows = (size_t)(K / every), first = (size_t)(b * K / every);
              if ((e = hipMemcpyAsync(thermo + first * ctx->R * kNQ, ctx->ring, rows * ctx->R * kNQ * sizeof(double),
                                      hipMemcpyDeviceToDevice, s)) != hipSuccess)
                return fail_hip(ctx, e);
            }
          }
          t_first = (int)(nblk * K) + 1;
        }
      }
      for (int t = t_first; t <= (persistent ? 0 : nsteps); ++t) {
        const bool rec = thermo && (t % thermo_every == 0);
        double* row = rec ? thermo + (size_t)(t / thermo_every - 1) * ctx->R * kNQ : nullptr;
        const bool timed = samples < max_samples && !rec && t % period == 0;
        KTimer tm_m, tm_f;
        if (timed) {
          tm_m = KTimer{ctx->tev[4 * samples], ctx->tev[4 * samples + 1]};
          tm_f = KTimer{ctx->tev[4 * samples + 2], ctx->tev[4 * samples + 3]};
          ++samples;
        }
        if ((e = enqueue_step(ctx, ph, lpa, t, nsteps, thermostat, rec, row, s, tm_m, tm_f)) != hipSuccess)
          return fail_hip(ctx, e);
      }
    }
    Flags fl;
    if ((e = read_flags(ctx, s, &fl)) != hipSuccess) return fail_hip(ctx, e);
    if (ctx->tune.persistent > 0 && nsteps > 0) ctx->last_groups = fl.pgroups;
    if (fl.abort) return SW_ETIMEOUT;
    if (fl.nbr_over || fl.cell_over) {
      if ((st = grow(ctx, fl)) != SW_OK) return st;
      continue;
    }
    const int par_final = nsteps & 1;
    if ((e = launch_scatter_out(ctx->d, par_final, (float4*)x, (float4*)v, (float4*)f, s)) != hipSuccess)
      return fail_hip(ctx, e);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail_hip(ctx, e);
    for (int k = 0; k < samples; ++k) {
      float a = 0.f, b = 0.f;
      if ((e = hipEventElapsedTime(&a, ctx->tev[4 * k], ctx->tev[4 * k + 1])) != hipSuccess) return fail_hip(ctx, e);
      if ((e = hipEventElapsedTime(&b, ctx->tev[4 * k + 2], ctx->tev[4 * k + 3])) != hipSuccess) return fail_hip(ctx, e);
      ctx->t_mom_ms += a;
      ctx->t_for_ms += b;
    }
    ctx->t_samples += samples;
    ctx->steps += nsteps;
    return fl.overlap ? SW_EOVERLAP : SW_OK;
  }
  return SW_ENBR_OVERFLOW;
}

int sw_query(sw_ctx* ctx, int what, long long* out) {
  if (!ctx || !out) return SW_EINVAL;
  switch (what) {
    case SW_Q_NATOMS: *out = ctx->N; return SW_OK;
    case SW_Q_NREPLICAS: *out = ctx->R; return SW_OK;
    case SW_Q_NBR_CAPACITY: *out = ctx->cap; return SW_OK;
    case SW_Q_CELL_CAPACITY: *out = ctx->cc; return SW_OK;
    case SW_Q_DEVICE_BYTES: *out = (long long)device_bytes(ctx); return SW_OK;
    case SW_Q_STEPS: *out = ctx->steps; return SW_OK;
    case SW_Q_TIME_MOMENTS_NS: *out = (long long)(ctx->t_mom_ms * 1e6); return SW_OK;
    case SW_Q_TIME_FORCES_NS: *out = (long long)(ctx->t_for_ms * 1e6); return SW_OK;
    case SW_Q_TIMED_STEPS: *out = ctx->t_samples; return SW_OK;
    case SW_Q_PERSISTENT_GROUPS: *out = ctx->last_groups; return SW_OK;
    case SW_Q_MIN_CELL_EDGE: {
      double m = 1e300;
      for (const RepInfo& R : ctx->reps)
        for (int k = 0; k < 3; ++k) m = std::min(m, R.L[k] / R.nc[k]);
      *out = (long long)std::floor(m * 1e6);
      return SW_OK;
    }
    case SW_Q_AUDIT_PAIRS:
    case SW_Q_MISSED_PAIRS: {
      unsigned long long h[2];
      hipError_t e = hipDeviceSynchronize();
      if (e == hipSuccess) e = hipMemcpy(h, ctx->d_audit, sizeof h, hipMemcpyDeviceToHost);
      if (e != hipSuccess) return fail_hip(ctx, e);
      *out = (long long)h[what == SW_Q_AUDIT_PAIRS ? 0 : 1];
      return SW_OK;
    }
    case SW_Q_REBUILDS: {
      int h[F_NFLAGS];
      hipError_t e = hipDeviceSynchronize();
      if (e == hipSuccess) e = hipMemcpy(h, ctx->d.flags, sizeof h, hipMemcpyDeviceToHost);
      if (e != hipSuccess) return fail_hip(ctx, e);
      *out = h[F_REBUILDS];
      return SW_OK;
    }
  }
  return SW_EINVAL;
}

}  // extern "C"
