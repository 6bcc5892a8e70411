// Isothermal-isobaric dynamics: host side of the Nose-Hoover thermostat and
// barostat of Sec. II.B (relaxation times tau_T, tau_P; the paper runs at
// p = 0), read as the isotropic Martyna-Tobias-Klein equations with
// Nose-Hoover chains.  The kernels are k_npt_kick (chains, barostat, first
// kick, scaled drift, binning), the moments kernel and the force kernel in
// its isobaric mode (second kick, kinetic and virial sums), then the
// per-replica reduction.  Every replica has its own box, temperature and
// pressure; boxes change every step, positions stay box fractions.
#include "sw_ctx.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

using namespace swk;
using namespace swh;

namespace {

constexpr double kGridMargin = 0.02;   // cell edges kept this much above cutoff + skin

NptState fresh_state(const sw_ctx* c, int r) {
  NptState s{};
  for (int k = 0; k < 3; ++k) s.L[k] = c->box[3 * r + k];
  return s;
}

int ensure_npt(sw_ctx* c) {
  hipError_t e;
  if (!c->d_npt &&
      (e = dalloc_raw(c, (void**)&c->d_npt, sizeof(NptState) * 2 * c->R, c->allocs)) != hipSuccess)
    return e == hipErrorOutOfMemory ? SW_ENOMEM : fail_hip(c, e);
  if (!c->d_nptc && (e = dalloc_raw(c, (void**)&c->d_nptc, sizeof(NptConst) * c->R, c->allocs)) != hipSuccess)
    return e == hipErrorOutOfMemory ? SW_ENOMEM : fail_hip(c, e);
  if (!c->npt_ready) {
    c->npt.resize(c->R);
    for (int r = 0; r < c->R; ++r) c->npt[r] = fresh_state(c, r);
    c->npt_ready = true;
  }
  return SW_OK;
}

// Box edges of the host view from the extended state (scales follow).
void set_boxes(sw_ctx* c, const std::vector<NptState>& st) {
  for (int r = 0; r < c->R; ++r)
    for (int k = 0; k < 3; ++k) {
      const double L = st[r].L[k];
      c->box[3 * r + k] = L;
      c->reps[r].L[k] = L;
      c->reps[r].scale[k] = (float)(L / kTwo32);
      c->reps[r].inv_scale[k] = (float)(kTwo32 / L);
    }
}

// Masses of the extended system for replica r (thermostat chain: Q_1 = N_f kT
// tau_T^2, later links kT tau_T^2; barostat W = (N_f + 3) kT tau_P^2 and its
// chain kT tau_P^2).
NptConst npt_const(const sw_ctx* c, int r, double T0, double p_ext, double tauT, double tauP) {
  NptConst k{};
  k.nf = 3.0 * c->reps[r].n - 3.0;
  k.kT = kBoltz * T0;
  k.alpha = 1.0 + 3.0 / k.nf;
  for (int j = 0; j < kNptChain; ++j) {
    k.Q[j] = (j == 0 ? k.nf : 1.0) * k.kT * tauT * tauT;
    k.iQ[j] = 1.0 / k.Q[j];
  }
  const bool baro = tauP > 0.0;
  k.Qb = baro ? k.kT * tauP * tauP : 1.0;
  k.iQb = 1.0 / k.Qb;
  k.Wb = baro ? (k.nf + 3.0) * k.kT * tauP * tauP : 1.0;
  k.iWb = 1.0 / k.Wb;
  k.pext = baro ? p_ext : 0.0;
  return k;
}

bool grid_fits(const sw_ctx* c, double margin) {
  const double rl = c->cutoff + c->skin;
  for (int r = 0; r < c->R; ++r)
    for (int k = 0; k < 3; ++k)
      if (c->box[3 * r + k] / c->reps[r].nc[k] < rl * (1.0 + margin)) return false;
  return true;
}

// One isobaric step t >= 2 (kick closing t-1 and opening t, moments, forces)
// with the launch arguments that depend on t; row_prev is the record of step
// t-1 or null, rec asks the moments launch for the energies of step t.
hipError_t enqueue_npt_step(sw_ctx* c, const Phys& ph, int lpa, int sums, NptArgs a, int t, double* row_prev, bool rec,
                            hipStream_t s) {
  a.in = c->d_npt + (size_t)((t - 1) & 1) * c->R;
  a.out = c->d_npt + (size_t)(t & 1) * c->R;
  a.mode = t == 1 ? NPT_BEGIN : NPT_STEP;
  a.par = (t - 1) & 1;
  a.row = row_prev;
  hipError_t e;
  if ((e = launch_npt_kick(c->d, ph, a, s)) != hipSuccess) return e;
  if ((e = launch_moments(c->d, ph, lpa, t & 1, 0, rec ? 1 : 0, s)) != hipSuccess) return e;
  return launch_forces(c->d, ph, lpa, MODE_NPT, sums, t & 1, nullptr, s);
}

// Captures steps 2 .. K+1 (K a multiple of 2 and of the record interval, so
// every later block t0+1 .. t0+K with t0 = 1 + b K has the same launch
// arguments) into a graph, records going to a ring of K / every rows,
// unless the cached graph matches.
hipError_t ensure_npt_graph(sw_ctx* c, const Phys& ph, int lpa, int sums, const NptArgs& tmpl, int K, int every) {
  std::vector<unsigned char> key(sizeof(Dev) + sizeof(Phys) + sizeof(NptArgs) + 5 * sizeof(int));
  const int meta[5] = {K, every, lpa, sums, c->alloc_gen};
  unsigned char* k = key.data();
  std::memcpy(k, &c->d, sizeof(Dev)); k += sizeof(Dev);
  std::memcpy(k, &ph, sizeof(Phys)); k += sizeof(Phys);
  std::memcpy(k, &tmpl, sizeof(NptArgs)); k += sizeof(NptArgs);
  std::memcpy(k, meta, sizeof meta);
  if (c->npt_gexec && key == c->npt_gkey) return hipSuccess;
  hipError_t e;
  if (c->npt_gexec) { (void)hipGraphExecDestroy(c->npt_gexec); c->npt_gexec = nullptr; }
  if (c->npt_graph) { (void)hipGraphDestroy(c->npt_graph); c->npt_graph = nullptr; }
  c->npt_gkey.clear();
  if (!c->cap_stream && (e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking)) != hipSuccess) return e;
  const size_t rows = every > 0 ? (size_t)(K / every) : 0;
  const size_t rowsz = (size_t)c->R * kNptRow;
  if (rows > c->npt_ring_rows) {
    if (c->npt_ring) (void)hipFree(c->npt_ring);
    c->npt_ring = nullptr;
    c->npt_ring_rows = 0;
    if ((e = hipMalloc((void**)&c->npt_ring, rows * rowsz * sizeof(double))) != hipSuccess) return e;
    c->npt_ring_rows = rows;
  }
  if ((e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
  hipError_t le = hipSuccess;
  for (int l = 1; l <= K && le == hipSuccess; ++l) {
    const int t = 1 + l;   // stands for t0 + l; steps l = t-1 with l % every == 0 are recorded
    double* row_prev = every > 0 && l % every == 0 ? c->npt_ring + (size_t)(l / every - 1) * rowsz : nullptr;
    le = enqueue_npt_step(c, ph, lpa, sums, tmpl, t, row_prev, every > 0 && t % every == 0, c->cap_stream);
  }
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(c->cap_stream, &g);
  if (le != hipSuccess) { if (g) (void)hipGraphDestroy(g); return le; }
  if (e != hipSuccess) return e;
  c->npt_graph = g;
  if ((e = hipGraphInstantiate(&c->npt_gexec, g, nullptr, nullptr, 0)) != hipSuccess) return e;
  c->npt_gkey = key;
  return hipSuccess;
}

}  // namespace

extern "C" {

int sw_npt(sw_ctx* ctx, float* x, float* v, float* f, const sw_params* params, double mass, double dt, int nsteps,
           const double* h_T0, const double* h_p_bar, double tau_T_fs, double tau_P_fs, int chain, int reset,
           double* rows, int every, void* stream) {
  if (!ctx || !x || !v || !h_T0 || !h_p_bar || nsteps < 0) return SW_EINVAL;
  if (!(tau_T_fs > 0.0) || !std::isfinite(tau_P_fs) || chain < 1 || chain > kNptChain) return SW_EINVAL;
  if (rows && every <= 0) return SW_EINVAL;
  for (int r = 0; r < ctx->R; ++r)
    if (!(h_T0[r] > 0.0) || !std::isfinite(h_T0[r]) || !std::isfinite(h_p_bar[r])) return SW_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  Phys ph{};
  int st = make_phys(ctx, params, mass, dt, &ph);
  if (st != SW_OK) return st;
  if ((st = ensure_npt(ctx)) != SW_OK) return st;
  if (reset)
    for (int r = 0; r < ctx->R; ++r) ctx->npt[r] = fresh_state(ctx, r);
  const std::vector<NptState> start = ctx->npt;
  std::vector<NptConst> cst(ctx->R);
  for (int r = 0; r < ctx->R; ++r) cst[r] = npt_const(ctx, r, h_T0[r], h_p_bar[r] * kBar, tau_T_fs, tau_P_fs);
  const std::vector<float2> unit(ctx->R, make_float2(1.f, 0.f));
  const int lpa = lpa_for(ctx);
  const double rl = ctx->cutoff + ctx->skin;
  // small replicas: the kick launch sums the force blocks' partials itself;
  // the force launches add a reduction launch only if some replica is larger
  const int apb = kBlock / lpa;
  const int sums = needs_reduce_launch(ctx->d, apb) ? 1 : 0;
  double margin = kGridMargin;
  set_boxes(ctx, start);
  if (!grid_fits(ctx, 0.5 * margin) && (st = regrid(ctx, margin)) != SW_OK) return st;
  int failure = SW_ENBR_OVERFLOW;
  for (int attempt = 0; attempt < 8; ++attempt) {
    hipError_t e;
    set_boxes(ctx, start);
    if ((e = hipMemcpyAsync(ctx->d_reps, ctx->reps.data(), sizeof(RepInfo) * ctx->R, hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(ctx->d_npt, start.data(), sizeof(NptState) * ctx->R, hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(ctx->d_nptc, cst.data(), sizeof(NptConst) * ctx->R, hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(ctx->d_T0, h_T0, sizeof(double) * ctx->R, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(ctx->d_kick, unit.data(), sizeof(float2) * ctx->R, hipMemcpyHostToDevice, s)) !=
            hipSuccess)
      return fail_hip(ctx, e);
    if ((e = reset_flags(ctx, s)) != hipSuccess) return fail_hip(ctx, e);
    if ((e = sort_in(ctx, x, v, s)) != hipSuccess) return fail_hip(ctx, e);
    // forces, virial and kinetic sums at the initial state (kick = identity)
    if ((e = launch_moments(ctx->d, ph, lpa, 0, 1, 0, s)) != hipSuccess) return fail_hip(ctx, e);
    if ((e = launch_forces(ctx->d, ph, lpa, MODE_NPT, sums, 0, nullptr, s)) != hipSuccess) return fail_hip(ctx, e);
    NptArgs a{};
    a.reps = ctx->d_reps;
    a.kick = ctx->d_kick;
    a.cst = ctx->d_nptc;
    a.tauT = tau_T_fs;
    a.tauP = tau_P_fs;
    a.rl = rl;
    a.rc = ctx->cutoff;
    a.dt = dt;
    a.c_m = kAcc / mass;
    a.chain = chain;
    a.apb = apb;
    const size_t rowsz = (size_t)ctx->R * kNptRow;
    auto row_of = [&](int step) -> double* {   // record of 1-based step, or null
      return rows && step > 0 && step % every == 0 ? rows + (size_t)(step / every - 1) * rowsz : nullptr;
    };
    // step 1 opens the trajectory; then captured blocks of K steps (t0 + 1 ..
    // t0 + K, t0 = 1 + b K) where the tuning asks for them; then the rest
    int t_next = 1;
    if (nsteps >= 1) {
      if ((e = enqueue_npt_step(ctx, ph, lpa, sums, a, 1, nullptr, row_of(1) != nullptr, s)) != hipSuccess)
        return fail_hip(ctx, e);
      t_next = 2;
    }
    if (ctx->tune.graph_steps > 0 && nsteps > 1) {
      const int ev = rows ? every : 0;
      long long period = 2;
      if (ev > 0) {
        long long x = period, y = ev;
        while (y) { const long long r = x % y; x = y; y = r; }
        period = period / x * ev;
      }
      const long long K = ((ctx->tune.graph_steps + period - 1) / period) * period;
      const long long nblk = (nsteps - 1) / K;
      if (nblk > 0 && K <= 1 << 20) {
        if ((e = ensure_npt_graph(ctx, ph, lpa, sums, a, (int)K, ev)) != hipSuccess) return fail_hip(ctx, e);
        for (long long b = 0; b < nblk; ++b) {
          if ((e = hipGraphLaunch(ctx->npt_gexec, s)) != hipSuccess) return fail_hip(ctx, e);
          if (ev > 0) {   // records of steps b K + ev .. (b + 1) K
            const size_t nr = (size_t)(K / ev), first = (size_t)(b * K / ev);
            if ((e = hipMemcpyAsync(rows + first * rowsz, ctx->npt_ring, nr * rowsz * sizeof(double),
                                    hipMemcpyDeviceToDevice, s)) != hipSuccess)
              return fail_hip(ctx, e);
          }
        }
        t_next = (int)(1 + nblk * K + 1);
      }
    }
    for (int t = t_next; t <= nsteps; ++t)
      if ((e = enqueue_npt_step(ctx, ph, lpa, sums, a, t, row_of(t - 1), row_of(t) != nullptr, s)) != hipSuccess)
        return fail_hip(ctx, e);
    if (nsteps > 0) {   // close the last step
      a.in = ctx->d_npt + (size_t)(nsteps & 1) * ctx->R;
      a.out = ctx->d_npt + (size_t)((nsteps + 1) & 1) * ctx->R;
      a.mode = NPT_END;
      a.par = nsteps & 1;
      a.row = row_of(nsteps);
      if ((e = launch_npt_kick(ctx->d, ph, a, s)) != hipSuccess) return fail_hip(ctx, e);
    }
    Flags fl;
    if ((e = read_flags(ctx, s, &fl)) != hipSuccess) return fail_hip(ctx, e);
    if (fl.nbr_over || fl.cell_over) {
      if ((st = grow(ctx, fl)) != SW_OK) return st;
      failure = SW_ENBR_OVERFLOW;
      continue;
    }
    std::vector<NptState> end(ctx->R);
    if ((e = hipMemcpy(end.data(), ctx->d_npt + (size_t)((nsteps + (nsteps > 0 ? 1 : 0)) & 1) * ctx->R,
                       sizeof(NptState) * ctx->R, hipMemcpyDeviceToHost)) != hipSuccess)
      return fail_hip(ctx, e);
    if (fl.box) {   // a box shrank below its cell grid: larger margin, redo the call
      set_boxes(ctx, start);
      margin *= 2.0;
      if ((st = regrid(ctx, margin)) != SW_OK) return st;
      failure = SW_EBOX_TOO_SMALL;
      continue;
    }
    if ((e = launch_scatter_out(ctx->d, nsteps & 1, (float4*)x, (float4*)v, (float4*)f, s)) != hipSuccess)
      return fail_hip(ctx, e);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail_hip(ctx, e);
    ctx->npt = end;
    set_boxes(ctx, end);
    if ((e = hipMemcpy(ctx->d_reps, ctx->reps.data(), sizeof(RepInfo) * ctx->R, hipMemcpyHostToDevice)) !=
        hipSuccess)
      return fail_hip(ctx, e);
    ctx->steps += nsteps;
    return fl.overlap ? SW_EOVERLAP : SW_OK;
  }
  set_boxes(ctx, start);
  return failure;
}

int sw_get_box(const sw_ctx* ctx, double* h_box) {
  if (!ctx || !h_box) return SW_EINVAL;
  std::memcpy(h_box, ctx->box.data(), sizeof(double) * 3 * ctx->R);
  return SW_OK;
}

int sw_npt_state(sw_ctx* ctx, double* h_state, int set) {
  if (!ctx || !h_state) return SW_EINVAL;
  int st = ensure_npt(ctx);
  if (st != SW_OK) return st;
  for (int r = 0; r < ctx->R; ++r) {
    double* o = h_state + (size_t)r * SW_NPT_STATE;
    NptState& n = ctx->npt[r];
    if (set) {
      n.ve = o[0];
      for (int k = 0; k < kNptChain; ++k) {
        n.xi[k] = o[1 + k]; n.vxi[k] = o[5 + k]; n.eta[k] = o[9 + k]; n.veta[k] = o[13 + k];
      }
    } else {
      o[0] = n.ve;
      for (int k = 0; k < kNptChain; ++k) {
        o[1 + k] = n.xi[k]; o[5 + k] = n.vxi[k]; o[9 + k] = n.eta[k]; o[13 + k] = n.veta[k];
      }
    }
  }
  return SW_OK;
}

}  // extern "C"
