// Structural observables of Sec. II.C of the mW paper on the device: the pair
// distance histogram behind g(r) and n_c, the angular distribution of each
// molecule's n_c closest neighbours, P(theta), and the unwrapped displacement
// behind the Einstein relation for D.
//
// Histograms are exact: distances and angles are formed in FP64 from the
// uint32 box fractions with single correctly rounded operations in a fixed
// order (the _rn intrinsics keep the compiler from fusing them), bins come
// from the caller's edge table by comparison, and counts are integer sums.
// Any implementation that follows the same coordinate convention and
// operation order gets the same counts.
//
// Each atom is handled by a group of 32 lanes; lane c < 27 walks cell c of
// the atom's 3x3x3 neighbourhood of binning cells, so the search radius is
// limited to the smallest cell edge of the replica.
#include "sw_ctx.h"
#include "sw_device.h"

#include <algorithm>
#include <cmath>

namespace swk {
namespace {

constexpr int kObsLPA = 32;
constexpr int kObsAPB = kBlock / kObsLPA;
constexpr int kObsMaxBins = 8192;
constexpr int kAdfCap = 64;        // neighbours inside the search radius kept per centre
constexpr int kAdfMaxNear = 16;

// Minimum-image difference of two atoms in FP64 (exact int -> double, one
// rounded product per component).
__device__ __forceinline__ void diff_f64(const uint4& a, const uint4& b, const RepInfo& R, double d[3]) {
  d[0] = __dmul_rn((double)(int)(b.x - a.x), R.L[0] / kTwo32);
  d[1] = __dmul_rn((double)(int)(b.y - a.y), R.L[1] / kTwo32);
  d[2] = __dmul_rn((double)(int)(b.z - a.z), R.L[2] / kTwo32);
}

__device__ __forceinline__ double dot_f64(const double a[3], const double b[3]) {
  return __dadd_rn(__dadd_rn(__dmul_rn(a[0], b[0]), __dmul_rn(a[1], b[1])), __dmul_rn(a[2], b[2]));
}

// Number of interior edges e[1..nb-1] (ascending) that are <= v.
__device__ __forceinline__ int count_le(const double* e, int nb, double v) {
  int lo = 1, hi = nb;   // answer + 1 in [lo, hi]
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (e[mid] <= v) lo = mid + 1;
    else hi = mid;
  }
  return lo - 1;
}

// Number of interior edges c[1..nb-1] (descending) that are >= v.
__device__ __forceinline__ int count_ge(const double* c, int nb, double v) {
  int lo = 1, hi = nb;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (c[mid] >= v) lo = mid + 1;
    else hi = mid;
  }
  return lo - 1;
}

// The binning cell of the atom's neighbourhood that lane c < 27 walks.
__device__ __forceinline__ int nbr_cell(const uint4& u, const RepInfo& R, int c) {
  const int n0 = R.nc[0], n1 = R.nc[1], n2 = R.nc[2];
  int xx = (int)__umulhi(u.x, (unsigned)n0) + c / 9 - 1;
  int yy = (int)__umulhi(u.y, (unsigned)n1) + (c / 3) % 3 - 1;
  int zz = (int)__umulhi(u.z, (unsigned)n2) + c % 3 - 1;
  xx += xx < 0 ? n0 : (xx >= n0 ? -n0 : 0);
  yy += yy < 0 ? n1 : (yy >= n1 ? -n1 : 0);
  zz += zz < 0 ? n2 : (zz >= n2 ? -n2 : 0);
  return R.cell_off + (xx * n1 + yy) * n2 + zz;
}

__device__ void flush_hist(const unsigned* hist, int nb, unsigned long long* out) {
  for (int b = threadIdx.x; b < nb; b += kBlock)
    if (hist[b]) atomicAdd(out + b, (unsigned long long)hist[b]);
}

// Ordered-pair counts per squared-distance bin, per replica.
__global__ __launch_bounds__(kBlock) void k_rdf(Dev d, const double* __restrict__ e, int nb,
                                                unsigned long long* __restrict__ counts) {
  extern __shared__ unsigned hist[];
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int g = threadIdx.x / kObsLPA, lane = threadIdx.x % kObsLPA;
  const int i = bid * kObsAPB + g;
  const int rep = d.tile_rep[(bid * kObsAPB) >> 6];
  const RepInfo& R = d.reps[rep];
  for (int b = threadIdx.x; b < nb; b += kBlock) hist[b] = 0u;
  __syncthreads();
  if (i < R.iend && lane < 27) {
    const uint4 ui = d.u[0][i];
    const int cell = nbr_cell(ui, R, lane);
    const int cnt = min(d.gcnt[0][cell], d.cc);
    const double lo = e[0], hi = e[nb];
    for (int s = 0; s < cnt; ++s) {
      const uint4 uj = d.gmem[0][(size_t)cell * d.cc + s];
      if ((int)uj.w == i) continue;
      double dd[3];
      diff_f64(ui, uj, R, dd);
      const double r2 = dot_f64(dd, dd);
      if (r2 >= lo && r2 < hi) atomicAdd(&hist[count_le(e, nb, r2)], 1u);
    }
  }
  __syncthreads();
  flush_hist(hist, nb, counts + (size_t)rep * nb);
}

// Angle counts over the n_near closest neighbours (by r^2, then caller
// index) inside the search radius of every centre, per replica.
__global__ __launch_bounds__(kBlock) void k_adf(Dev d, int n_near, double rs2, const double* __restrict__ c, int nb,
                                                unsigned long long* __restrict__ counts,
                                                unsigned long long* __restrict__ flags) {
  extern __shared__ unsigned hist[];
  __shared__ double cr2[kObsAPB][kAdfCap];
  __shared__ double cd[kObsAPB][kAdfCap][3];
  __shared__ int cid[kObsAPB][kAdfCap];
  __shared__ int ncand[kObsAPB];
  __shared__ int sel[kObsAPB][kAdfMaxNear];
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int g = threadIdx.x / kObsLPA, lane = threadIdx.x % kObsLPA;
  const int i = bid * kObsAPB + g;
  const int rep = d.tile_rep[(bid * kObsAPB) >> 6];
  const RepInfo& R = d.reps[rep];
  const bool real = i < R.iend;
  for (int b = threadIdx.x; b < nb; b += kBlock) hist[b] = 0u;
  if (lane == 0) ncand[g] = 0;
  __syncthreads();
  if (real && lane < 27) {
    const uint4 ui = d.u[0][i];
    const int cell = nbr_cell(ui, R, lane);
    const int cnt = min(d.gcnt[0][cell], d.cc);
    for (int s = 0; s < cnt; ++s) {
      const uint4 uj = d.gmem[0][(size_t)cell * d.cc + s];
      if ((int)uj.w == i) continue;
      double dd[3];
      diff_f64(ui, uj, R, dd);
      const double r2 = dot_f64(dd, dd);
      if (r2 < rs2) {
        const int k = atomicAdd(&ncand[g], 1);
        if (k < kAdfCap) {
          cr2[g][k] = r2;
          cid[g][k] = d.ids[uj.w];
          cd[g][k][0] = dd[0]; cd[g][k][1] = dd[1]; cd[g][k][2] = dd[2];
        }
      }
    }
  }
  __syncthreads();
  const int n = min(ncand[g], kAdfCap);
  if (real && lane == 0 && ncand[g] > kAdfCap) atomicAdd(flags + 1, 1ull);
  const bool ok = real && ncand[g] <= kAdfCap && n >= n_near;
  if (real && lane == 0 && ncand[g] <= kAdfCap && n < n_near) atomicAdd(flags, 1ull);
  if (ok) {
    // rank of each candidate in (r^2, caller index) order; the first n_near are kept
    for (int k = lane; k < n; k += kObsLPA) {
      int rank = 0;
      for (int q = 0; q < n; ++q)
        rank += cr2[g][q] < cr2[g][k] || (cr2[g][q] == cr2[g][k] && cid[g][q] < cid[g][k]);
      if (rank < n_near) sel[g][rank] = k;
    }
  }
  __syncthreads();
  if (ok) {
    const int npair = n_near * (n_near - 1) / 2;
    for (int p = lane; p < npair; p += kObsLPA) {
      int a = 0, rest = p;
      while (rest >= n_near - 1 - a) {
        rest -= n_near - 1 - a;
        ++a;
      }
      const int b = a + 1 + rest;
      const int ka = sel[g][a], kb = sel[g][b];
      const double dot = dot_f64(cd[g][ka], cd[g][kb]);
      const double cs = __ddiv_rn(dot, __dsqrt_rn(__dmul_rn(cr2[g][ka], cr2[g][kb])));
      atomicAdd(&hist[count_ge(c, nb, cs)], 1u);
    }
  }
  __syncthreads();
  flush_hist(hist, nb, counts + (size_t)rep * nb);
}

// Unwrapped displacement in caller order: acc += minimum image of (x - last).
__global__ void k_msd_update(const float4* __restrict__ x, long long n, const long long* __restrict__ uoff, int R,
                             const RepInfo* __restrict__ reps, double* __restrict__ last, double* __restrict__ acc,
                             int reset) {
  const long long k = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  int lo = 0, hi = R - 1;   // replica of caller atom k
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (uoff[mid] <= k) lo = mid;
    else hi = mid - 1;
  }
  const float4 p = x[k];
  const double xs[3] = {(double)p.x, (double)p.y, (double)p.z};
  for (int c = 0; c < 3; ++c) {
    const size_t o = (size_t)3 * k + c;
    if (reset) {
      acc[o] = 0.0;
    } else {
      const double L = reps[lo].L[c];
      double dd = __dsub_rn(xs[c], last[o]);
      dd = __dsub_rn(dd, __dmul_rn(L, rint(__ddiv_rn(dd, L))));
      acc[o] = __dadd_rn(acc[o], dd);
    }
    last[o] = xs[c];
  }
}

// Mean square displacement per replica: one block per replica, fixed order.
__global__ __launch_bounds__(kBlock) void k_msd_reduce(const long long* __restrict__ uoff, int R,
                                                       const double* __restrict__ acc, double* __restrict__ msd) {
  __shared__ double tree[kBlock];
  for (int r = blockIdx.x; r < R; r += gridDim.x) {
    double s = 0.0;
    for (long long k = uoff[r] + threadIdx.x; k < uoff[r + 1]; k += kBlock) {
      const double* a = acc + 3 * k;
      s += (a[0] * a[0] + a[1] * a[1]) + a[2] * a[2];
    }
    tree[threadIdx.x] = s;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st) tree[threadIdx.x] += tree[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const long long n = uoff[r + 1] - uoff[r];
      msd[r] = n > 0 ? tree[0] / (double)n : 0.0;
    }
    __syncthreads();
  }
}

}  // namespace
}  // namespace swk

using namespace swk;
using namespace swh;

namespace {

hipError_t obs_alloc(sw_ctx* c) {
  hipError_t e;
  if (!c->obs_edges &&
      (e = dalloc_raw(c, (void**)&c->obs_edges, sizeof(double) * (kObsMaxBins + 1), c->allocs)) != hipSuccess)
    return e;
  if (!c->obs_flags &&
      (e = dalloc_raw(c, (void**)&c->obs_flags, sizeof(unsigned long long) * 2, c->allocs)) != hipSuccess)
    return e;
  return hipSuccess;
}

// Smallest binning-cell edge over the replicas: the search radius limit.
double min_cell_edge(const sw_ctx* c) {
  double m = 1e300;
  for (const RepInfo& R : c->reps)
    for (int k = 0; k < 3; ++k) m = std::min(m, R.L[k] / R.nc[k]);
  return m;
}

// Sort and bin the caller's positions (grid 0); grows the cell capacity and
// redoes the binning if a cell overflowed.
int bin_positions(sw_ctx* c, const float* x, hipStream_t s) {
  for (int attempt = 0; attempt < 6; ++attempt) {
    hipError_t e;
    if ((e = reset_flags(c, s)) != hipSuccess) return fail_hip(c, e);
    if ((e = sort_in(c, x, nullptr, s)) != hipSuccess) return fail_hip(c, e);
    c->have_order = false;   // the new internal order no longer matches the rows
    Flags fl;
    if ((e = read_flags(c, s, &fl)) != hipSuccess) return fail_hip(c, e);
    if (!fl.cell_over) return SW_OK;
    Flags only{0, 0, 1, 0, 0};
    int st = grow(c, only);
    if (st != SW_OK) return st;
  }
  return SW_ECELL_OVERFLOW;
}

}  // namespace

extern "C" {

int sw_rdf(sw_ctx* ctx, const float* x, int nbins, const double* h_r2_edges, unsigned long long* counts,
           void* stream) {
  if (!ctx || !x || !h_r2_edges || !counts || nbins < 1 || nbins > kObsMaxBins) return SW_EINVAL;
  for (int k = 0; k < nbins; ++k)
    if (!(h_r2_edges[k] < h_r2_edges[k + 1])) return SW_EINVAL;
  if (!(h_r2_edges[0] >= 0.0)) return SW_EINVAL;
  const double rc = min_cell_edge(ctx);
  if (!(h_r2_edges[nbins] <= rc * rc)) return SW_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if ((e = obs_alloc(ctx)) != hipSuccess) return fail_hip(ctx, e);
  int st = bin_positions(ctx, x, s);
  if (st != SW_OK) return st;
  if ((e = hipMemcpyAsync(ctx->obs_edges, h_r2_edges, sizeof(double) * (nbins + 1), hipMemcpyHostToDevice, s)) !=
      hipSuccess)
    return fail_hip(ctx, e);
  if ((e = hipMemsetAsync(counts, 0, sizeof(unsigned long long) * ctx->R * nbins, s)) != hipSuccess)
    return fail_hip(ctx, e);
  hipLaunchKernelGGL(k_rdf, dim3((unsigned)(ctx->npad / kObsAPB)), dim3(kBlock), sizeof(unsigned) * nbins, s,
                     ctx->d, (const double*)ctx->obs_edges, nbins, counts);
  if ((e = hipGetLastError()) != hipSuccess) return fail_hip(ctx, e);
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail_hip(ctx, e);
  return SW_OK;
}

int sw_adf(sw_ctx* ctx, const float* x, int n_near, double r_search, int nbins, const double* h_cos_edges,
           unsigned long long* counts, long long* h_short, void* stream) {
  if (!ctx || !x || !h_cos_edges || !counts || nbins < 1 || nbins > kObsMaxBins) return SW_EINVAL;
  if (n_near < 2 || n_near > kAdfMaxNear || !(r_search > 0.0) || !(r_search <= min_cell_edge(ctx))) return SW_EINVAL;
  for (int k = 0; k < nbins; ++k)
    if (!(h_cos_edges[k] > h_cos_edges[k + 1])) return SW_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if ((e = obs_alloc(ctx)) != hipSuccess) return fail_hip(ctx, e);
  int st = bin_positions(ctx, x, s);
  if (st != SW_OK) return st;
  if ((e = hipMemcpyAsync(ctx->obs_edges, h_cos_edges, sizeof(double) * (nbins + 1), hipMemcpyHostToDevice, s)) !=
      hipSuccess)
    return fail_hip(ctx, e);
  if ((e = hipMemsetAsync(counts, 0, sizeof(unsigned long long) * ctx->R * nbins, s)) != hipSuccess)
    return fail_hip(ctx, e);
  if ((e = hipMemsetAsync(ctx->obs_flags, 0, sizeof(unsigned long long) * 2, s)) != hipSuccess)
    return fail_hip(ctx, e);
  hipLaunchKernelGGL(k_adf, dim3((unsigned)(ctx->npad / kObsAPB)), dim3(kBlock), sizeof(unsigned) * nbins, s,
                     ctx->d, n_near, r_search * r_search, (const double*)ctx->obs_edges, nbins, counts,
                     ctx->obs_flags);
  if ((e = hipGetLastError()) != hipSuccess) return fail_hip(ctx, e);
  unsigned long long fl[2] = {0, 0};
  if ((e = hipMemcpyAsync(fl, ctx->obs_flags, sizeof fl, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return fail_hip(ctx, e);
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail_hip(ctx, e);
  if (h_short) *h_short = (long long)fl[0];
  return fl[1] ? SW_ENBR_OVERFLOW : SW_OK;
}

int sw_msd(sw_ctx* ctx, const float* x, int reset, double* msd, void* stream) {
  if (!ctx || !x || !msd) return SW_EINVAL;
  if (!reset && !ctx->msd_ready) return SW_ESTATE;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  const size_t n3 = (size_t)3 * std::max<long long>(ctx->N, 1);
  for (double** p : {&ctx->msd_last, &ctx->msd_acc}) {
    if (!*p && (e = dalloc_raw(ctx, (void**)p, sizeof(double) * n3, ctx->allocs)) != hipSuccess)
      return fail_hip(ctx, e);
  }
  if (ctx->N > 0)
    hipLaunchKernelGGL(k_msd_update, dim3((unsigned)((ctx->N + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       (const float4*)x, ctx->N, (const long long*)ctx->d_uoff, ctx->R,
                       (const RepInfo*)ctx->d_reps, ctx->msd_last, ctx->msd_acc, reset ? 1 : 0);
  hipLaunchKernelGGL(k_msd_reduce, dim3((unsigned)std::min(ctx->R, 4096)), dim3(kBlock), 0, s,
                     (const long long*)ctx->d_uoff, ctx->R, (const double*)ctx->msd_acc, msd);
  if ((e = hipGetLastError()) != hipSuccess) return fail_hip(ctx, e);
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail_hip(ctx, e);
  ctx->msd_ready = true;
  return SW_OK;
}

}  // extern "C"
