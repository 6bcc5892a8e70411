// HIP kernels of the mW Stillinger-Weber engine for gfx950 (MI355X).
//
// Model: Eq. E of Sec. II.A (pair term phi2 plus the three-body term phi3 with
// its vertex at the centre atom), parameters of Sec. II.A / II.D.
//
// The three-body energy of centre i is evaluated from per-centre moments.
// With e_j = exp(gamma sigma / (r_ij - a sigma)), unit vectors u_j and
// c0 = cos(theta0):
//   T = sum_j e_j u_j u_j^T,  V = sum_j e_j u_j,  S = sum_j e_j,  P = sum_j e_j^2
//   sum_{j<k} e_j e_k (u_j.u_k - c0)^2 = 1/2 [ |T|_F^2 - 2 c0 |V|^2 + c0^2 S^2 - (1-c0)^2 P ]
// an exact identity (the diagonal j = k terms are removed by the P term), so
// E3_i = lambda eps times the bracket.  Its gradient with respect to the leg
// vector d_j = r_j u_j is
//   G_j = lambda eps e_j [ g_j q_j u_j + (2/r_j) (I - u_j u_j^T)(T u_j - c0 V) ]
//   q_j = u_j^T T u_j - 2 c0 V.u_j + c0^2 S - e_j (1-c0)^2,  g_j = -gamma sigma/(r_j - a sigma)^2
// The force on atom m gathers its own centre's G (with + sign) and minus the
// G of every neighbour centre i evaluated on the leg i->m, so each atom writes
// only its own force: no atomics, deterministic sums.  One moments kernel and
// one force kernel make a step; the force kernel also integrates.
//
// Positions are unsigned 32-bit fractions of the box edge: the minimum image
// of a difference is its two's-complement value, exact for any box size.

#include "sw_internal.h"
#include "sw_device.h"

#include <hip/hip_ext.h>

namespace swk {
namespace {

// Replica geometry the integrator needs, read into registers before the
// kernel's first store (later reads could not be hoisted above the stores).
struct Geo {
  float sc0, sc1, sc2, is0, is1, is2;
  int nc0, nc1, nc2, cell_off;
};

__device__ __forceinline__ Geo geo_of(const RepInfo& R) {
  return Geo{R.scale[0], R.scale[1], R.scale[2], R.inv_scale[0], R.inv_scale[1], R.inv_scale[2],
             R.nc[0], R.nc[1], R.nc[2], R.cell_off};
}

// Drift by tx*v in fraction units (tx = dt, or its isobaric equivalent),
// store the new position in buffer `gp`, and raise the replica's rebuild
// flag if the atom is now more than hs (half the effective skin) away from
// its row-build position.  Flags steps longer than a quarter edge.  Returns
// the atom's cell in grid `gp`; u becomes the new position.
__device__ __forceinline__ int drift(const Dev& d, const Geo& G, int rep, int i, uint4& u, const float4& v,
                                     const uint4& uref, float tx, float hs, int gp) {
  const float mx = tx * v.x * G.is0;
  const float my = tx * v.y * G.is1;
  const float mz = tx * v.z * G.is2;
  const float lim = 1073741824.0f;  // 2^30: a quarter of the edge
  if (!(fabsf(mx) < lim && fabsf(my) < lim && fabsf(mz) < lim)) atomicOr(&d.flags[F_OVERLAP], 2);
  u.x += (unsigned)__float2int_rn(fminf(fmaxf(mx, -lim), lim));
  u.y += (unsigned)__float2int_rn(fminf(fmaxf(my, -lim), lim));
  u.z += (unsigned)__float2int_rn(fminf(fmaxf(mz, -lim), lim));
  const float3 dd = disp(uref, u, G.sc0, G.sc1, G.sc2);
  const bool moved = dd.x * dd.x + dd.y * dd.y + dd.z * dd.z > hs * hs;
  pick(d.u, gp)[i] = u;
  if (moved) d.dflag[gp * d.R + rep] = 1;
  return G.cell_off + cell_of(u, G.nc0, G.nc1, G.nc2);
}

// Appends entry e (position, index in .w) to cell c of grid `gp`.
__device__ __forceinline__ void cell_put(const Dev& d, int gp, int c, const uint4& e) {
  const int slot = atomicAdd(&pick(d.gcnt, gp)[c], 1);
  if (slot < d.cc) pick(d.gmem, gp)[(size_t)c * d.cc + slot] = e;
  else atomicOr(&d.flags[F_CELL_OVER], 1);
}

// As cell_put for the wavefront's binned entries (lanes with c >= 0), with
// one counter atomic per distinct cell of the wavefront.  Used where every
// lane bins an atom (the thermostat kernel) in large contexts: atoms are in
// Morton order, so consecutive lanes often share a cell (the replica table:
// 112.8 -> 109.3 us per step).  In small contexts, in the force kernel (one
// binning lane per group) and in the isobaric kick the extra pass measured
// slower than one atomic per atom.
// Every lane of the wavefront calls it (lanes with nothing to bin pass
// c = -1).  The order of entries within a cell is not fixed; rows are sorted
// when built.
__device__ __forceinline__ void cell_append(const Dev& d, int gp, int c, const uint4& e) {
  const int lane = (int)__lane_id();
  unsigned long long todo = __ballot(c >= 0);
  int leader = lane, rank = 0, count = 0;
  while (todo) {   // one pass per distinct cell, uniform
    const int src = __ffsll((unsigned long long)todo) - 1;
    const int cc = __builtin_amdgcn_readlane(c, src);
    const unsigned long long same = __ballot(c == cc) & todo;
    if ((same >> lane) & 1ull) {
      leader = src;
      rank = __popcll(same & ((1ull << lane) - 1ull));
    }
    if (lane == src) count = __popcll(same);
    todo &= ~same;
  }
  int base = 0;
  if (count > 0) base = atomicAdd(&pick(d.gcnt, gp)[c], count);
  base = __shfl(base, leader, 64);
  if (c >= 0) {
    const int slot = base + rank;
    if (slot < d.cc) pick(d.gmem, gp)[(size_t)c * d.cc + slot] = e;
    else atomicOr(&d.flags[F_CELL_OVER], 1);
  }
}

// ----------------------------------------------------------------- sorting
__global__ __launch_bounds__(kBlock) void k_sort_count(const float4* __restrict__ x, long long n,
                                                      const long long* __restrict__ uoff, int R,
                                                      const RepInfo* __restrict__ reps,
                                                      const int* __restrict__ cell_rank,
                                                      uint4* __restrict__ uq, int* __restrict__ key,
                                                      int* __restrict__ cnt) {
  const long long k = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  int lo = 0, hi = R - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (uoff[mid] <= k) lo = mid; else hi = mid - 1;
  }
  const RepInfo& Rp = reps[lo];
  const float4 p = x[k];
  const uint4 u = make_uint4(quantize(p.x, 1.0 / Rp.L[0]), quantize(p.y, 1.0 / Rp.L[1]),
                             quantize(p.z, 1.0 / Rp.L[2]), 0u);
  const int rank = cell_rank[Rp.cell_off + cell_of(u, Rp.nc[0], Rp.nc[1], Rp.nc[2])];
  uq[k] = u;
  key[k] = rank;
  atomicAdd(&cnt[rank], 1);
}

// Exclusive scan of n counts with one block of 1024 threads.  Each thread
// owns a contiguous range, read 16 counts per batch of independent loads
// (a thread's one-at-a-time loop waited on every load: 121 us for the
// 68921 cells of the 262144-atom box).
constexpr int kScanBatch = 16;

__global__ __launch_bounds__(1024) void k_scan(const int* __restrict__ cnt, int* __restrict__ start, int n) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int b = min(n, t * per), e = min(n, b + per);
  int s = 0;
  for (int k0 = b; k0 < e; k0 += kScanBatch) {
    int v[kScanBatch];
#pragma unroll
    for (int u = 0; u < kScanBatch; ++u) v[u] = k0 + u < e ? cnt[k0 + u] : 0;
#pragma unroll
    for (int u = 0; u < kScanBatch; ++u) s += v[u];
  }
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int add = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  int run = part[t] - s;
  for (int k0 = b; k0 < e; k0 += kScanBatch) {
    int v[kScanBatch];
#pragma unroll
    for (int u = 0; u < kScanBatch; ++u) v[u] = k0 + u < e ? cnt[k0 + u] : 0;
#pragma unroll
    for (int u = 0; u < kScanBatch; ++u)
      if (k0 + u < e) {
        start[k0 + u] = run;
        run += v[u];
      }
  }
}

__global__ __launch_bounds__(kBlock) void k_sort_scatter(long long n, const int* __restrict__ key,
                                                        const int* __restrict__ start, int* __restrict__ cursor,
                                                        int* __restrict__ order) {
  const long long k = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  const int r = key[k];
  order[start[r] + atomicAdd(&cursor[r], 1)] = (int)k;
}

// Within each cell, order atoms by caller index so the layout is deterministic.
__global__ __launch_bounds__(kBlock) void k_sort_cells(int ncell, const int* __restrict__ cnt,
                                                      const int* __restrict__ start, int* __restrict__ order) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= ncell) return;
  const int b = start[c], m = cnt[c];
  for (int a = 1; a < m; ++a) {
    const int v = order[b + a];
    int q = a - 1;
    while (q >= 0 && order[b + q] > v) {
      order[b + q + 1] = order[b + q];
      --q;
    }
    order[b + q + 1] = v;
  }
}

__global__ __launch_bounds__(kBlock) void k_gather_sorted(Dev d, const uint4* __restrict__ uq,
                                                         const float4* __restrict__ v_user,
                                                         const int* __restrict__ order) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= d.npad) return;
  const RepInfo& R = d.reps[d.tile_rep[i >> 6]];
  const int local = i - R.ioff;
  if (local < R.n) {
    const int k = order[R.uoff + local];
    d.ids[i] = k;
    d.u[0][i] = uq[k];
    float4 vv = v_user ? v_user[k] : make_float4(0.f, 0.f, 0.f, 0.f);
    vv.w = 0.f;
    d.v[i] = vv;
  } else {
    d.ids[i] = -1;
    d.u[0][i] = make_uint4(0u, 0u, 0u, 0u);
    d.u[1][i] = make_uint4(0u, 0u, 0u, 0u);
    d.v[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    d.f[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    d.uref[i] = make_uint4(0u, 0u, 0u, 0u);
    d.nn[i] = 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_gather_ids(Dev d, const float4* __restrict__ x_user, int par) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= d.npad) return;
  const int k = d.ids[i];
  if (k < 0) return;
  const RepInfo& R = d.reps[d.tile_rep[i >> 6]];
  const float4 p = x_user[k];
  d.u[par][i] = make_uint4(quantize(p.x, 1.0 / R.L[0]), quantize(p.y, 1.0 / R.L[1]),
                           quantize(p.z, 1.0 / R.L[2]), 0u);
}

// Bin positions u[par] into grid `par` (counts must be zero) and, if asked,
// raise the replica's rebuild flag for atoms that moved too far from their
// row-build position.  Rows hold every atom within rl of the build position
// in the box of that build (edge lref); a box scaled since then (isobaric
// steps) scales those distances by s = L / lref, so an atom may move
// (s rl - rc) / 2 in the current box before a pair inside rc can be missing.
__global__ __launch_bounds__(kBlock) void k_bin(Dev d, int par, int check, float rl, float rc) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < d.npad) {
    const int rep = d.tile_rep[i >> 6];
    const RepInfo& R = d.reps[rep];
    if (i < R.iend) {
      const uint4 u = d.u[par][i];
      const int c = R.cell_off + cell_of(u, R.nc[0], R.nc[1], R.nc[2]);
      const int slot = atomicAdd(&d.gcnt[par][c], 1);
      if (slot < d.cc) d.gmem[par][(size_t)c * d.cc + slot] = make_uint4(u.x, u.y, u.z, (unsigned)i);
      else atomicOr(&d.flags[F_CELL_OVER], 1);
      if (check) {
        const float hs = (float)(0.5 * (R.L[0] / d.lref[rep] * rl - rc) - 1e-4);
        const float3 dd = disp(d.uref[i], u, R.scale[0], R.scale[1], R.scale[2]);
        if (!(hs > 0.f) || dd.x * dd.x + dd.y * dd.y + dd.z * dd.z > hs * hs) d.dflag[par * d.R + rep] = 1;
      }
    }
  }
}

// ----------------------------------------------------------------- moments
// One group of LPA lanes per atom.  When the replica's displacement flag (or
// the caller) asks for it, the group first rebuilds the atom's row from the
// 27 surrounding binning cells (each cell stores positions with the atom
// index in .w, so a cell is one contiguous read), keeping every atom within
// cutoff + skin, sorted by index.  Then the group accumulates T, V, S (and
// P, E2 on energy steps) over the active neighbours r < a sigma.
// Clears the cell counts and displacement flags of the other parity; every
// block of a moments launch (or phase) takes a grid-stride share.
__device__ __forceinline__ void clear_next(const Dev& d, int par, int b, int G, unsigned tid) {
  for (int r = b * kBlock + tid; r < d.R; r += G * kBlock) d.dflag[(par ^ 1) * d.R + r] = 0;
  for (int c = b * kBlock + tid; c < d.ctot; c += G * kBlock) pick(d.gcnt, par ^ 1)[c] = 0;
}

// The group's candidate count, and INT_MAX in the slots past it up to a
// multiple of four (the capacity is one), so the sort reads whole quads.
__device__ __forceinline__ void pad_count(int* cand, int* cnt, int run, int cap) {
  *cnt = run;
  const int t = min(run, cap);
  for (int z = t; z < ((t + 3) & ~3); ++z) cand[z] = 0x7fffffff;
}

// lds: [APB][cs] candidates, [APB][cs] sorted (cs = lds_row_stride(APB, cap)
// >= cap), [APB] counts, [APB][56] cell prefix and ids; with 16 or more lanes
// per atom also [APB][cap] candidate positions (16-byte aligned)
template <int LPA, bool ENERGY, bool TAN = false>
__device__ void moments_tile(const Dev& d, const Phys& p, int par, int force_rebuild, int bid, unsigned tid, int* lds,
                             const float4* __restrict__ tw = nullptr, float4* __restrict__ tmd = nullptr) {
  constexpr int APB = kBlock / LPA;
  // row slots per lane per batch: a batch spans at most 32 slots, one
  // 128-byte line of the row; with 8 lanes per atom 24 slots, which hold the
  // ~16-entry rows of a 0.5 A skin (a wavefront issues every slot of a batch,
  // used or not)
  constexpr int kMU = LPA == 8 ? 3 : (LPA >= 32 ? 1 : (32 / LPA < 4 ? 32 / LPA : 4));
  const int g = tid / LPA, lane = tid % LPA;
  const int i = bid * APB + g;
  // Every load that does not depend on another is issued up front, before
  // the kernel's first store: own position, row length and the first batch
  // of row slots (slots below the capacity are always addressable; they are
  // masked by the row length later; the atom arrays are padded to npad, so
  // padding atoms read in bounds too), and the tile's replica (a per-lane
  // load that joins the batch; a context of one replica needs none).  Then
  // the replica's geometry and rebuild flag.
  const int cap = d.cap;
  const int* row = d.nl + (size_t)i * cap;
  const uint4 ui = pick(d.u, par)[i];
  int jn[kMU];
#pragma unroll
  for (int u = 0; u < kMU; ++u) jn[u] = row[min(lane + u * LPA, cap - 1)];
  const int nn_all = d.nn[i];
  const int rep = d.R == 1 ? 0 : __builtin_amdgcn_readfirstlane(d.tile_rep[i >> 6]);
  const RepInfo& R = d.reps[rep];
  const Geo G = geo_of(R);
  const int iend = R.iend, ioff = R.ioff;
  const float sc0 = G.sc0, sc1 = G.sc1, sc2 = G.sc2;
  const bool real = i < iend;
  const int nn_row = real ? nn_all : 0;
  // each replica rebuilds on its own displacement record, or (sync_rb) all
  // replicas when any record is set: one lane per replica, then a ballot
  bool flagged;
  if (d.sync_rb) {
    int f = 0;
    for (int r = (tid & 63); r < d.R; r += 64) f |= d.dflag[par * d.R + r];
    flagged = __ballot(f != 0) != 0ull;
  } else {
    flagged = d.dflag[par * d.R + rep] != 0;
  }
  const bool rebuild = force_rebuild || flagged;
  int nn = nn_row;
  bool from_lds = false;                   // row slots name candidate positions in LDS
  const uint4* lds_u = nullptr;

  if (rebuild) {                           // block-uniform
    const int cs = lds_row_stride(APB, cap);         // per-atom stride of the two lists (>= cap)
    int* cand = lds + g * cs;
    int* srt = lds + APB * cs + g * cs;
    int* cnt = lds + 2 * APB * cs;
    int* pre = lds + 2 * APB * cs + APB + g * 56;    // [28] prefix of cell counts
    // candidate positions (16+ lanes per atom): the moments below read the
    // rebuilt row's neighbour positions from here instead of gathering them
    uint4* cand_u = reinterpret_cast<uint4*>(
                        reinterpret_cast<char*>(lds) + ((sizeof(int) * moments_lds_ints(APB, cap) + 15) & ~(size_t)15)) +
                    g * cap;
    int* cid = pre + 28;                             // [27] cell ids
    if (lane == 0) cnt[g] = 0;
    const int n0 = G.nc0, n1 = G.nc1, n2 = G.nc2;
    const int cx = (int)__umulhi(ui.x, (unsigned)n0);
    const int cy = (int)__umulhi(ui.y, (unsigned)n1);
    const int cz = (int)__umulhi(ui.z, (unsigned)n2);
    const int* gc = pick(d.gcnt, par);
    const uint4* gm = pick(d.gmem, par);
    const int ccap = d.cc;
    // Lane l owns the contiguous cells [l*CPL, (l+1)*CPL): their counts are
    // one batch of loads, and a prefix scan over the group gives every
    // cell's prefix.  Neighbouring atoms read the same cells, so these reads
    // and the candidate reads below mostly hit the CU's L1.
    constexpr int CPL = (27 + LPA - 1) / LPA;
    int cl[CPL], mc[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int c = min(lane * CPL + q, 26);     // lanes past the 27 cells read cell 26, masked below
      int xx = cx + c / 9 - 1, yy = cy + (c / 3) % 3 - 1, zz = cz + c % 3 - 1;
      xx = xx < 0 ? xx + n0 : (xx >= n0 ? xx - n0 : xx);
      yy = yy < 0 ? yy + n1 : (yy >= n1 ? yy - n1 : yy);
      zz = zz < 0 ? zz + n2 : (zz >= n2 ? zz - n2 : zz);
      cl[q] = G.cell_off + (xx * n1 + yy) * n2 + zz;
      mc[q] = gc[cl[q]];
    }
    // An unconditional use of every count keeps the compiler from sinking
    // the loads into the masking branches below, which would serialise them.
#pragma unroll
    for (int q = 0; q < CPL; ++q) asm volatile("" ::"v"(mc[q]));
#pragma unroll
    for (int q = 0; q < CPL; ++q) mc[q] = (real && lane * CPL + q < 27) ? min(mc[q], ccap) : 0;
    int own = 0;
#pragma unroll
    for (int q = 0; q < CPL; ++q) own += mc[q];
    const int incl = group_prefix<LPA>(own, lane);   // inclusive scan of the lanes' totals
    // With fewer than 16 lanes per atom (and a row capacity that holds it),
    // the candidate -> cell lookup is a rank: bit p of a 256-bit mask marks
    // the first candidate of a non-empty cell, and the r-th non-empty cell's
    // entry base sits in a table, so candidate k < 256 reads entry
    // base[rank(k)] + k, with rank(k) = (set bits at or below k) - 1.  Both
    // live in the sorted-row area, unused until the sort.  Mask words and
    // their prefix counts interleave: msk[2w] = word w, msk[2w + 1] = bits
    // set in the words below w.
    constexpr bool kRankLookup = LPA < 16;
    const bool rank_ok = kRankLookup && cs >= kRankInts;
    int* msk = srt;
    int* cbase = srt + 16;
    if (real) {
      int run = incl - own;
      int ne = 0;
      if (rank_ok) {
#pragma unroll
        for (int q = 0; q < CPL; ++q) ne += mc[q] > 0;
        for (int w = lane; w < 8; w += LPA) msk[2 * w] = 0;
      }
      int nrank = group_prefix<LPA>(ne, lane) - ne;    // non-empty cells of the lanes below
      if (lane == 0) pre[0] = 0;
#pragma unroll
      for (int q = 0; q < CPL; ++q) {
        const int c = lane * CPL + q;
        if (rank_ok && mc[q] > 0) {
          if (run < 256) atomicOr(reinterpret_cast<unsigned*>(&msk[2 * (run >> 5)]), 1u << (run & 31));
          cbase[nrank++] = (int)((unsigned)cl[q] * (unsigned)ccap - (unsigned)run);   // mod 2^32, like at below
        }
        run += mc[q];
        if (c < 27) {
          pre[c + 1] = run;
          cid[c] = cl[q];
        }
      }
    }
    __syncthreads();
    if (real && rank_ok) {
      // exclusive prefix of the mask words' bit counts (words [lane * WPL, +WPL))
      constexpr int WPL = kRankLookup ? 8 / LPA : 1;
      int pc[WPL], tot = 0;
#pragma unroll
      for (int j = 0; j < WPL; ++j) {
        pc[j] = __builtin_popcount((unsigned)msk[2 * (lane * WPL + j)]);
        tot += pc[j];
      }
      int ex = group_prefix<LPA>(tot, lane) - tot;
#pragma unroll
      for (int j = 0; j < WPL; ++j) {
        msk[2 * (lane * WPL + j) + 1] = ex;
        ex += pc[j];
      }
    }
    __syncthreads();
    if (real && LPA >= 16) {
      // Many lanes per atom (small boxes, few waves in flight: latency
      // bound).  The cell of every candidate slot of a pass is found by a
      // branch-free binary search (the largest c with pre[c] <= k) run for
      // all the pass's slots level by level, one LDS round trip per level;
      // steps past cell 26 read pre[27] = ncand, which no slot reaches, and
      // slots past the end search for the last candidate and are rejected.
      // Accepted entries are compacted with a ballot over the group.
      const int ncand = pre[27];
      const float rl2 = p.rl2;
      const int wl = tid & 63;
      const unsigned long long gmask = LPA == 64 ? ~0ull : ((1ull << LPA) - 1) << (wl & ~(LPA - 1));
      const unsigned long long below = (1ull << wl) - 1;
      int run = 0;                             // entries appended so far (lane 0 sees every pass)
      constexpr int kCL = 6;
      for (int k0 = lane; k0 < ncand; k0 += kCL * LPA) {
        int c[kCL];
#pragma unroll
        for (int t = 0; t < kCL; ++t) c[t] = 0;
#pragma unroll
        for (int step = 16; step >= 1; step >>= 1) {
#pragma unroll
          for (int t = 0; t < kCL; ++t) {
            const int nc = c[t] + step;
            c[t] = pre[min(nc, 27)] <= min(k0 + t * LPA, ncand - 1) ? nc : c[t];
          }
        }
        uint4 e[kCL];
#pragma unroll
        for (int t = 0; t < kCL; ++t)
          e[t] = gm[(size_t)cid[c[t]] * ccap + (min(k0 + t * LPA, ncand - 1) - pre[c[t]])];
#pragma unroll
        for (int t = 0; t < kCL; ++t) {
          const int j = (int)e[t].w;
          const float3 dd = disp(ui, e[t], sc0, sc1, sc2);
          const bool acc = k0 + t * LPA < ncand && j != i && dd.x * dd.x + dd.y * dd.y + dd.z * dd.z < rl2;
          const unsigned long long m = __ballot(acc) & gmask;
          if (acc) {
            const int sl = run + __popcll(m & below);
            if (sl < cap) {
              cand[sl] = j;
              cand_u[sl] = e[t];   // a cell entry holds the position of that parity
            }
          }
          run += __popcll(m);
        }
      }
      if (lane == 0) pad_count(cand, cnt + g, run, cap);
    } else if (real) {
      // Few lanes per atom (large boxes, the CU full of waves: bound by
      // instruction issue).  Each slot finds its cell entry on its own (the
      // rank lookup above, else a binary search over the cell prefix) and
      // skips the load past the end; entry indices are 32-bit, and accepted
      // entries are compacted with a group ballot (no LDS atomics).
      const int ncand = pre[27];
      const float rl2 = p.rl2;
      const int wl = tid & 63;
      const int gsh = wl & ~(LPA - 1);                           // the group's first lane
      // (this branch runs with fewer than 16 lanes per atom; the mask is
      // spelled so that every instantiation compiles)
      constexpr unsigned gmk = LPA < 32 ? (1u << (LPA % 32)) - 1u : ~0u;
      const unsigned gbl = (1u << (wl - gsh)) - 1u;
      int run = 0;                                               // entries appended so far (group-uniform)
      constexpr int kCL = 8;
      auto scan = [&](auto entry_at) {
        for (int k0 = lane; k0 < ncand; k0 += kCL * LPA) {
          uint4 e[kCL];
#pragma unroll
          for (int t = 0; t < kCL; ++t) {
            const int k = k0 + t * LPA;
            e[t] = make_uint4(ui.x, ui.y, ui.z, (unsigned)i);
            if (k < ncand) e[t] = gm[entry_at(k)];
          }
#pragma unroll
          for (int t = 0; t < kCL; ++t) {
            const int j = (int)e[t].w;
            const float3 dd = disp(ui, e[t], sc0, sc1, sc2);
            const bool acc = j != i && dd.x * dd.x + dd.y * dd.y + dd.z * dd.z < rl2;
            const unsigned m = (unsigned)(__ballot(acc) >> gsh) & gmk;
            if (acc) {
              const int sl = run + __builtin_popcount(m & gbl);
              if (sl < cap) cand[sl] = j;
            }
            run += __builtin_popcount(m);
          }
        }
      };
      // group-uniform choice; the search covers atoms with over 256 candidates
      if (rank_ok && ncand <= 256) {
        scan([&](int k) -> unsigned {
          const int w = k >> 5;
          const unsigned bits = (unsigned)msk[2 * w] & ((2u << (k & 31)) - 1u);
          return (unsigned)cbase[msk[2 * w + 1] + __builtin_popcount(bits) - 1] + (unsigned)k;
        });
      } else {
        scan([&](int k) -> unsigned {
          int c = 0;
#pragma unroll
          for (int step = 16; step >= 1; step >>= 1)
            if (c + step < 27 && pre[c + step] <= k) c += step;
          return (unsigned)cid[c] * (unsigned)ccap + (unsigned)(k - pre[c]);
        });
      }
      if (lane == 0) pad_count(cand, cnt + g, run, cap);
    }
    __syncthreads();
    int total = cnt[g];
    if (real && lane == 0 && total > cap) {
      atomicOr(&d.flags[F_NBR_OVER], 1);
      atomicMax(&d.flags[F_NBR_NEED], total);
    }
    total = min(total, cap);
    if (real) {
      // Ascending neighbour index: the row and every later sum over it are
      // independent of the order the cells were filled in.  With candidate
      // positions in LDS the sorted list holds candidate slots, else indices.
      // The list is read four entries at a time (16-byte aligned; the
      // entries past the count up to a multiple of four hold INT_MAX).
      const int4* cand4 = reinterpret_cast<const int4*>(cand);
      for (int k = lane; k < total; k += LPA) {
        const int vj = cand[k];
        int rank = 0;
#pragma unroll 1
        for (int q = 0; q < total; q += 4) {
          const int4 w = cand4[q >> 2];
          rank += (w.x < vj) + (w.y < vj) + (w.z < vj) + (w.w < vj);
        }
        srt[rank] = (LPA >= 16 && !TAN) ? k : vj;
        d.nl[(size_t)i * cap + rank] = vj;
      }
      if (lane == 0) {
        d.nn[i] = total;
        d.uref[i] = ui;
      }
    }
    __syncthreads();
    nn = real ? total : 0;
    row = srt;
    if (LPA >= 16 && !TAN) {   // the tangent mode gathers by atom index (it also reads w[j])
      from_lds = true;
      lds_u = cand_u;
    }
#pragma unroll
    for (int u = 0; u < kMU; ++u) jn[u] = srt[min(lane + u * LPA, cap - 1)];
    if (bid * APB == ioff && tid == 0) {
      atomicAdd(&d.flags[F_REBUILDS], 1);
      d.lref[rep] = R.L[0];
    }
  }

  float T0 = 0.f, T1 = 0.f, T2 = 0.f, T3 = 0.f, T4 = 0.f, T5 = 0.f;
  float V0 = 0.f, V1 = 0.f, V2 = 0.f, S = 0.f, P = 0.f, E2 = 0.f;
  // tangent mode: the moments' derivatives along the direction w as well
  // (the dual-number arithmetic of the tangent kernels, same per-lane order);
  // with tw null, along a uniform scaling of every leg (each leg's tangent is
  // the leg itself)
  float dT0 = 0.f, dT1 = 0.f, dT2 = 0.f, dT3 = 0.f, dT4 = 0.f, dT5 = 0.f, dV0 = 0.f, dV1 = 0.f, dV2 = 0.f, dS = 0.f;
  const float4 wi = TAN && tw ? tw[i] : make_float4(0.f, 0.f, 0.f, 0.f);
  const uint4* upm = pick(d.u, par);
  // With 8 or fewer lanes per atom the entries within the cutoff are also
  // written out, in row order, as the force kernel's row: a row holds ~40 %
  // more entries than the cutoff sphere, and the force loop then runs one
  // batch of slots instead of two.  The order follows from a group ballot per
  // slot batch (a lane that leaves the loop early has no entry left).
  constexpr bool kAct = LPA <= 8;
  int* act_row = d.act + (size_t)i * cap;
  const int wla = tid & 63;
  const int ash = wla & ~(LPA - 1);                          // the group's first lane
  const unsigned amask = (1u << (kAct ? LPA : 1)) - 1u;      // its bits, shifted down
  const unsigned abelow = (1u << (wla - ash)) - 1u;          // lanes of the group below this one
  int nact = 0;
  // pipelined like the force loop: a batch of slots' positions, then the
  // arithmetic, with the next batch's slots read in between
  for (int s0 = lane; s0 < nn; s0 += kMU * LPA) {
    int jj[kMU];
#pragma unroll
    for (int u = 0; u < kMU; ++u) jj[u] = s0 + u * LPA < nn ? jn[u] : -1;
#pragma unroll
    for (int u = 0; u < kMU; ++u) jn[u] = row[min(s0 + (kMU + u) * LPA, nn - 1)];
    uint4 uu[kMU];
    float4 wu[kMU];
#pragma unroll
    for (int u = 0; u < kMU; ++u) {
      uu[u] = ui;
      wu[u] = wi;
      if (jj[u] >= 0) {
        if (from_lds) uu[u] = lds_u[jj[u]];
        else uu[u] = upm[jj[u]];
        if (TAN && tw) wu[u] = tw[jj[u]];
      }
    }
#pragma unroll
    for (int u = 0; u < kMU; ++u) {
      const float3 dd = disp(ui, uu[u], sc0, sc1, sc2);
      const float r2 = dd.x * dd.x + dd.y * dd.y + dd.z * dd.z;
      if (kAct) {
        const bool in = jj[u] >= 0 && r2 < p.rc2;
        const unsigned m = (unsigned)(__ballot(in) >> ash) & amask;
        if (in) act_row[nact + __builtin_popcount(m & abelow)] = jj[u];
        nact += __builtin_popcount(m);
      }
      if (jj[u] >= 0 && r2 < p.rc2) {
        const float ir = rsq(r2);
        const float ux = dd.x * ir, uy = dd.y * ir, uz = dd.z * ir;
        const float idr = rcp(r2 * ir - p.rc);
        const float eg = ex2(p.gsig_l2e * idr);
        const float ex = eg * ux, ey = eg * uy, ez = eg * uz;
        T0 += ex * ux; T1 += ey * uy; T2 += ez * uz;
        T3 += ex * uy; T4 += ex * uz; T5 += ey * uz;
        V0 += ex; V1 += ey; V2 += ez; S += eg;
        if (ENERGY) {
          P += eg * eg;
          const float e1 = ex2(p.sig_l2e * idr);
          const float sr = p.sig * ir, s2 = sr * sr;
          E2 += 0.5f * p.Aeps * (p.B * s2 * s2 - 1.f) * e1;
        }
        if (TAN) {
          const Leg L = leg_dual(dd, tw ? sub3(wu[u], wi) : dd, p);
          const D dx = L.eg * L.ux, dy = L.eg * L.uy, dz = L.eg * L.uz;
          dT0 += (dx * L.ux).d; dT1 += (dy * L.uy).d; dT2 += (dz * L.uz).d;
          dT3 += (dx * L.uy).d; dT4 += (dx * L.uz).d; dT5 += (dy * L.uz).d;
          dV0 += dx.d; dV1 += dy.d; dV2 += dz.d; dS += L.eg.d;
        }
      }
    }
  }
  T0 = group_sum<LPA>(T0); T1 = group_sum<LPA>(T1); T2 = group_sum<LPA>(T2);
  T3 = group_sum<LPA>(T3); T4 = group_sum<LPA>(T4); T5 = group_sum<LPA>(T5);
  V0 = group_sum<LPA>(V0); V1 = group_sum<LPA>(V1); V2 = group_sum<LPA>(V2);
  S = group_sum<LPA>(S);
  float E3 = 0.f;
  if (ENERGY) {
    P = group_sum<LPA>(P);
    E2 = group_sum<LPA>(E2);
    const float tn2 = T0 * T0 + T1 * T1 + T2 * T2 + 2.f * (T3 * T3 + T4 * T4 + T5 * T5);
    const float vn2 = V0 * V0 + V1 * V1 + V2 * V2;
    E3 = 0.5f * p.lameps * (tn2 - 2.f * p.c0 * vn2 + p.c0 * p.c0 * S * S - p.qc * P);
  }
  if (real && lane == 0) {
    float4* m = d.mom + 3 * (size_t)i;
    m[0] = make_float4(T0, T1, T2, T3);
    m[1] = make_float4(T4, T5, V0, V1);
    m[2] = make_float4(V2, S, E2, E3);
    if (kAct) d.nact[i] = nact;
  }
  if (TAN) {
    dT0 = group_sum<LPA>(dT0); dT1 = group_sum<LPA>(dT1); dT2 = group_sum<LPA>(dT2);
    dT3 = group_sum<LPA>(dT3); dT4 = group_sum<LPA>(dT4); dT5 = group_sum<LPA>(dT5);
    dV0 = group_sum<LPA>(dV0); dV1 = group_sum<LPA>(dV1); dV2 = group_sum<LPA>(dV2);
    dS = group_sum<LPA>(dS);
    if (real && lane == 0) {
      float4* m = tmd + 3 * (size_t)i;
      m[0] = make_float4(dT0, dT1, dT2, dT3);
      m[1] = make_float4(dT4, dT5, dV0, dV1);
      m[2] = make_float4(dV2, dS, 0.f, 0.f);
    }
  }
}

template <int LPA, bool ENERGY>
__global__ __launch_bounds__(kBlock) void k_moments(Dev d, Phys p, int par, int force_rebuild) {
  extern __shared__ int lds[];
  moments_tile<LPA, ENERGY>(d, p, par, force_rebuild, xcd_remap(blockIdx.x, gridDim.x), threadIdx.x, lds);
  clear_next(d, par, blockIdx.x, gridDim.x, threadIdx.x);
}

// Moments with energies and their tangent along w: the primal moments of
// k_moments and the tangent moments of the tangent pass in one launch.
template <int LPA>
__global__ __launch_bounds__(kBlock) void k_moments_tan(Dev d, Phys p, int par, int force_rebuild,
                                                        const float4* __restrict__ w, float4* __restrict__ mdot) {
  extern __shared__ int lds[];
  moments_tile<LPA, true, true>(d, p, par, force_rebuild, xcd_remap(blockIdx.x, gridDim.x), threadIdx.x, lds, w,
                                mdot);
  clear_next(d, par, blockIdx.x, gridDim.x, threadIdx.x);
}

// ----------------------------------------------------------------- audit
// Missed-pair audit: one lane per atom walks the 27 cells of grid par (the
// binning of the positions this step reads), and for every j within the
// cut-off (the same float test as the moments kernel) looks j up in the
// atom's row by bisection (rows are ascending).  Counts go to two 64-bit
// counters, one atomic per wavefront each.
__global__ __launch_bounds__(kBlock) void k_audit(Dev d, Phys p, int par, unsigned long long* __restrict__ counts) {
  const int i = blockIdx.x * kBlock + (int)threadIdx.x;
  if (i >= d.npad) return;                             // whole wavefronts
  const int rep = d.tile_rep[i >> 6];
  const RepInfo& R = d.reps[rep];
  unsigned long long seen = 0, missed = 0;
  if (i < R.iend) {
    const uint4 ui = pick(d.u, par)[i];
    const int n0 = R.nc[0], n1 = R.nc[1], n2 = R.nc[2];
    const int cx = (int)__umulhi(ui.x, (unsigned)n0);
    const int cy = (int)__umulhi(ui.y, (unsigned)n1);
    const int cz = (int)__umulhi(ui.z, (unsigned)n2);
    const int* gc = pick(d.gcnt, par);
    const uint4* gm = pick(d.gmem, par);
    const int* row = d.nl + (size_t)i * d.cap;
    const int nn = d.nn[i];
    for (int c = 0; c < 27; ++c) {
      int xx = cx + c / 9 - 1, yy = cy + (c / 3) % 3 - 1, zz = cz + c % 3 - 1;
      xx = xx < 0 ? xx + n0 : (xx >= n0 ? xx - n0 : xx);
      yy = yy < 0 ? yy + n1 : (yy >= n1 ? yy - n1 : yy);
      zz = zz < 0 ? zz + n2 : (zz >= n2 ? zz - n2 : zz);
      const int cell = R.cell_off + (xx * n1 + yy) * n2 + zz;
      const int m = min(gc[cell], d.cc);
      for (int r = 0; r < m; ++r) {
        const uint4 e = gm[(size_t)cell * d.cc + r];
        const int j = (int)e.w;
        const float3 dd = disp(ui, e, R.scale[0], R.scale[1], R.scale[2]);
        if (j == i || !(dd.x * dd.x + dd.y * dd.y + dd.z * dd.z < p.rc2)) continue;
        ++seen;
        int lo = 0, hi = nn;                           // first slot with row[slot] >= j
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (row[mid] < j) lo = mid + 1;
          else hi = mid;
        }
        if (lo == nn || row[lo] != j) ++missed;
      }
    }
  }
  for (int o = 32; o >= 1; o >>= 1) {
    seen += __shfl_xor(seen, o, 64);
    missed += __shfl_xor(missed, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&counts[0], seen);
    if (missed) atomicAdd(&counts[1], missed);
  }
}

// ----------------------------------------------------------------- forces
// Block partial sums of the thermo quantities (fixed order within the block).
// The per-replica sums are taken by k_reduce_thermo after the kernel ends.
template <int APB>
__device__ void block_partials(const Dev& d, int bid, const double* q, bool writer, int g, unsigned tid) {
  static_assert(APB >= kMinAPB, "partial sums are sized for at least kMinAPB atoms per block");
  __shared__ double red[APB * kNQ];
  if (writer) {
#pragma unroll
    for (int k = 0; k < kNQ; ++k) red[g * kNQ + k] = q[k];
  }
  __syncthreads();
  if (tid < kNQ) {
    double acc = 0.0;
    for (int a = 0; a < APB; ++a) acc += red[a * kNQ + tid];
    d.partial[(size_t)tid * (d.npad / APB) + bid] = acc;
  }
  __syncthreads();   // red[] is reused by the block's next tile
}

// Force on each atom from its neighbours (pair term + its own centre's
// three-body term + the legs of the neighbour centres), then, by mode:
//   FORCES   store F (and thermo sums)
//   START    v += dt/2 a; drift
//   NVE      v += dt/2 a (full step: KE); v += dt/2 a; drift
//   NVE_LAST v += dt/2 a (full step: KE)
//   KICK     as NVE_LAST, the thermostat kernel follows
template <int LPA, int MODE, bool VIR>
__device__ void forces_tile(const Dev& d, const Phys& p, int par, int bid, unsigned tid) {
  constexpr int APB = kBlock / LPA;
  const int g = tid / LPA, lane = tid % LPA;
  const int i = bid * APB + g;
  // Software pipelined.  Everything that does not depend on a previous load
  // is issued first as one batch: own position, moments and row length, the
  // first kFU row slots of every lane (read whatever the row length, since
  // slots below the capacity are always addressable, and masked once it is
  // known), the velocity and row-build position the integrator needs, and
  // the tile's replica (a per-lane load, so it joins the batch; a context of
  // one replica needs none).  The atom arrays are padded to npad, so these
  // reads are in bounds for padding atoms too, whose values are masked.
  // Then, per kFU slots, the neighbours' positions and moments are one batch
  // of independent loads before any arithmetic.  The per-lane order of
  // neighbours is the plain stride order.
  constexpr int kFU = LPA >= 32 ? 1 : 2;   // a batch spans at most 32 slots (one row line)
  constexpr bool kAct = LPA <= 8;          // the moments launch's rows of entries within the cutoff
  const int cap = d.cap;
  const int* row = (kAct ? d.act : d.nl) + (size_t)i * cap;
  const uint4* up = pick(d.u, par);
  const uint4 ui = up[i];
  const float4* m = d.mom + 3 * (size_t)i;
  const float4 ma = m[0], mb = m[1], mc = m[2];
  const int nn_row = kAct ? d.nact[i] : d.nn[i];
  int jn[kFU];
#pragma unroll
  for (int u = 0; u < kFU; ++u) jn[u] = row[min(lane + u * LPA, cap - 1)];
  const float4 vi = MODE != MODE_FORCES ? d.v[i] : make_float4(0.f, 0.f, 0.f, 0.f);
  const uint4 urefi = (MODE == MODE_START || MODE == MODE_NVE) ? d.uref[i] : make_uint4(0u, 0u, 0u, 0u);
  const int rep = d.R == 1 ? 0 : __builtin_amdgcn_readfirstlane(d.tile_rep[i >> 6]);
  const RepInfo& R = d.reps[rep];
  const Geo G = geo_of(R);
  const float sc0 = G.sc0, sc1 = G.sc1, sc2 = G.sc2;
  const bool real = i < R.iend;
  const float c0 = p.c0, c02 = p.c0 * p.c0;

  float Tm0 = 0.f, Tm1 = 0.f, Tm2 = 0.f, Tm3 = 0.f, Tm4 = 0.f, Tm5 = 0.f, Vm0 = 0.f, Vm1 = 0.f, Vm2 = 0.f,
        Sm = 0.f, E2i = 0.f, E3i = 0.f;
  int nn = 0;
  if (real) {
    Tm0 = ma.x; Tm1 = ma.y; Tm2 = ma.z; Tm3 = ma.w; Tm4 = mb.x; Tm5 = mb.y;
    Vm0 = mb.z; Vm1 = mb.w; Vm2 = mc.x; Sm = mc.y; E2i = mc.z; E3i = mc.w;
    nn = nn_row;
  }
  float fx = 0.f, fy = 0.f, fz = 0.f;
  float w0 = 0.f, w1 = 0.f, w2 = 0.f, w3 = 0.f, w4 = 0.f, w5 = 0.f;
  for (int s0 = lane; s0 < nn; s0 += kFU * LPA) {
    int jj[kFU];
#pragma unroll
    for (int u = 0; u < kFU; ++u) {
      const int s = s0 + u * LPA;
      jj[u] = s < nn ? jn[u] : -1;
    }
#pragma unroll
    for (int u = 0; u < kFU; ++u) jn[u] = row[min(s0 + (kFU + u) * LPA, nn - 1)];   // next batch's slots
    uint4 uu[kFU];
    float4 mja[kFU], mjb[kFU], mjc[kFU];
#pragma unroll
    for (int u = 0; u < kFU; ++u) {
      if (jj[u] >= 0) {
        const float4* mj = d.mom + 3 * (size_t)jj[u];
        uu[u] = up[jj[u]];
        mja[u] = mj[0]; mjb[u] = mj[1]; mjc[u] = mj[2];
      } else {
        uu[u] = ui;
      }
    }
    float3 ddv[kFU];
    float r2v[kFU];
    bool act[kFU];
#pragma unroll
    for (int u = 0; u < kFU; ++u) {
      ddv[u] = disp(ui, uu[u], sc0, sc1, sc2);
      r2v[u] = ddv[u].x * ddv[u].x + ddv[u].y * ddv[u].y + ddv[u].z * ddv[u].z;
      act[u] = jj[u] >= 0 && r2v[u] < p.rc2;
    }
#pragma unroll
    for (int u = 0; u < kFU; ++u) {
    if (act[u]) {
      const int j = jj[u];
      const float3 dd = ddv[u];
      const float r2 = r2v[u];
      if (r2 < 0.25f) atomicOr(&d.flags[F_OVERLAP], 1);
      const float ir = rsq(r2);
      const float r = r2 * ir;
      const float ux = dd.x * ir, uy = dd.y * ir, uz = dd.z * ir;
      const float idr = rcp(r - p.rc);
      const float idr2 = idr * idr;
      const float e1 = ex2(p.sig_l2e * idr);
      const float eg = ex2(p.gsig_l2e * idr);
      const float sr = p.sig * ir, s4 = (sr * sr) * (sr * sr);
      const float poly = p.B * s4 - 1.f;
      const float dphi = p.Aeps * e1 * (-4.f * p.B * s4 * ir - poly * p.sig * idr2);
      const float gg = -p.gsig * idr2;
      (void)j;
      const float4 na = mja[u], nb = mjb[u], nc = mjc[u];
      const float Ts0 = Tm0 + na.x, Ts1 = Tm1 + na.y, Ts2 = Tm2 + na.z, Ts3 = Tm3 + na.w;
      const float Ts4 = Tm4 + nb.x, Ts5 = Tm5 + nb.y;
      const float Dv0 = Vm0 - nb.z, Dv1 = Vm1 - nb.w, Dv2 = Vm2 - nc.x, Ss = Sm + nc.y;
      const float y0x = Ts0 * ux + Ts3 * uy + Ts4 * uz;
      const float y0y = Ts3 * ux + Ts1 * uy + Ts5 * uz;
      const float y0z = Ts4 * ux + Ts5 * uy + Ts2 * uz;
      const float uTu = ux * y0x + uy * y0y + uz * y0z;
      const float uDv = ux * Dv0 + uy * Dv1 + uz * Dv2;
      const float q = uTu - 2.f * c0 * uDv + c02 * Ss - 2.f * p.qc * eg;
      const float uy_ = uTu - c0 * uDv;
      const float px = (y0x - c0 * Dv0) - uy_ * ux;
      const float py = (y0y - c0 * Dv1) - uy_ * uy;
      const float pz = (y0z - c0 * Dv2) - uy_ * uz;
      const float le = p.lameps * eg;
      const float a1 = dphi + le * gg * q;
      const float a2 = 2.f * le * ir;
      fx += a1 * ux + a2 * px;
      fy += a1 * uy + a2 * py;
      fz += a1 * uz + a2 * pz;
      if (VIR) {
        const float ymx = Tm0 * ux + Tm3 * uy + Tm4 * uz - c0 * Vm0;
        const float ymy = Tm3 * ux + Tm1 * uy + Tm5 * uz - c0 * Vm1;
        const float ymz = Tm4 * ux + Tm5 * uy + Tm2 * uz - c0 * Vm2;
        const float uym = ux * ymx + uy * ymy + uz * ymz;                 // u.(T u) - c0 u.V
        const float uVm = ux * Vm0 + uy * Vm1 + uz * Vm2;
        const float qown = uym - c0 * uVm + c02 * Sm - p.qc * eg;         // u.T.u - 2 c0 u.V + ...
        const float pox = ymx - uym * ux, poy = ymy - uym * uy, poz = ymz - uym * uz;
        const float cA = -(0.5f * r * dphi + le * r * gg * qown);
        const float cB = -2.f * le;
        w0 += cA * ux * ux + cB * ux * pox;
        w1 += cA * uy * uy + cB * uy * poy;
        w2 += cA * uz * uz + cB * uz * poz;
        w3 += cA * ux * uy + cB * ux * poy;
        w4 += cA * ux * uz + cB * ux * poz;
        w5 += cA * uy * uz + cB * uy * poz;
      }
    }
    }
  }
  fx = group_sum<LPA>(fx); fy = group_sum<LPA>(fy); fz = group_sum<LPA>(fz);
  if (VIR) {
    w0 = group_sum<LPA>(w0); w1 = group_sum<LPA>(w1); w2 = group_sum<LPA>(w2);
    w3 = group_sum<LPA>(w3); w4 = group_sum<LPA>(w4); w5 = group_sum<LPA>(w5);
  }

  constexpr bool kReduce = VIR || MODE == MODE_KICK || MODE == MODE_NPT;
  double q[kNQ];
#pragma unroll
  for (int k = 0; k < kNQ; ++k) q[k] = 0.0;
  if (real && lane == 0) {
    const float4 F = make_float4(fx, fy, fz, 0.f);
    d.f[i] = F;
    if (VIR) {
      q[0] = E2i; q[1] = E3i;
      q[3] = w0; q[4] = w1; q[5] = w2; q[6] = w3; q[7] = w4; q[8] = w5;
    }
    if (MODE == MODE_NPT) {
      const float2 k = d.npt_kick[rep];
      float4 v = vi;
      v.x = k.x * v.x + k.y * F.x; v.y = k.x * v.y + k.y * F.y; v.z = k.x * v.z + k.y * F.z;
      const float vx2 = v.x * v.x, vy2 = v.y * v.y, vz2 = v.z * v.z;
      q[2] = (double)(p.half_m_acc * (vx2 + vy2 + vz2));
      q[9] = (double)(p.m_acc * vx2); q[10] = (double)(p.m_acc * vy2); q[11] = (double)(p.m_acc * vz2);
      d.v[i] = v;
    } else if (MODE != MODE_FORCES) {
      float4 v = vi;
      v.x += p.hdt_cm * F.x; v.y += p.hdt_cm * F.y; v.z += p.hdt_cm * F.z;
      if (MODE != MODE_START) {
        const float vx2 = v.x * v.x, vy2 = v.y * v.y, vz2 = v.z * v.z;
        q[2] = (double)(p.half_m_acc * (vx2 + vy2 + vz2));
        q[9] = (double)(p.m_acc * vx2); q[10] = (double)(p.m_acc * vy2); q[11] = (double)(p.m_acc * vz2);
      }
      if (MODE == MODE_NVE) {
        v.x += p.hdt_cm * F.x; v.y += p.hdt_cm * F.y; v.z += p.hdt_cm * F.z;
      }
      if (MODE == MODE_START || MODE == MODE_NVE) {
        uint4 un = ui;
        const int c = drift(d, G, rep, i, un, v, urefi, p.dt, p.half_skin, par ^ 1);
        cell_put(d, par ^ 1, c, make_uint4(un.x, un.y, un.z, (unsigned)i));
      }
      d.v[i] = v;
    }
  }
  if (kReduce) block_partials<APB>(d, bid, q, lane == 0, g, tid);
}

template <int LPA, int MODE, bool VIR>
__global__ __launch_bounds__(kBlock) void k_forces(Dev d, Phys p, int par) {
  forces_tile<LPA, MODE, VIR>(d, p, par, xcd_remap(blockIdx.x, gridDim.x), threadIdx.x);
}

// Per-replica sums of the block partials: one block per (replica, quantity),
// threads stride over the replica's blocks, then a fixed tree.
__device__ void reduce_task(const Dev& d, int apb, double* ring_row, int task, unsigned tid) {
  __shared__ double tree[kBlock];
  const int nbt = d.npad / apb;
  {
    const int rep = task / kNQ, k = task % kNQ;
    const RepInfo& R = d.reps[rep];
    const int b0 = R.ioff / apb, b1 = R.ipad_end / apb;
    const double* src = d.partial + (size_t)k * nbt;
    double acc = 0.0;
    for (int b = b0 + tid; b < b1; b += kBlock) acc += src[b];
    tree[tid] = acc;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
      if (tid < st) tree[tid] += tree[tid + st];
      __syncthreads();
    }
    if (tid == 0) {
      d.thermo_cur[rep * kNQ + k] = tree[0];
      if (ring_row) ring_row[rep * kNQ + k] = tree[0];
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_reduce_thermo(Dev d, int apb, double* ring_row) {
  for (int task = blockIdx.x; task < d.R * kNQ; task += gridDim.x) reduce_task(d, apb, ring_row, task, threadIdx.x);
}

// Sums over replica R of the force launch's block partials of quantities
// ks[0..nk) (nk <= 4), for a replica of at most kFusedBlocks blocks of apb
// atoms.  Every wave of the replica takes them in one fixed order: one
// batch of loads, lane-strided sums, then a butterfly, which leaves the same
// bits in every lane, so all waves of the replica hold identical totals.
// All 64 lanes of the wave must call it.
__device__ __forceinline__ void replica_sums(const Dev& d, int apb, const RepInfo& R, const int (&ks)[4], int nk,
                                             double* out, unsigned tid) {
  constexpr int kJ = kFusedBlocks / 64;
  const int lane = tid & 63;
  const int nbt = d.npad / apb, b0 = R.ioff / apb, b1 = R.ipad_end / apb;
  double x[4][kJ];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int j = 0; j < kJ; ++j)
      x[q][j] = q < nk ? d.partial[(size_t)ks[q] * nbt + min(b0 + lane + 64 * j, b1 - 1)] : 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < kJ; ++j)
      if (b0 + lane + 64 * j < b1) acc += x[q][j];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (q < nk) out[ks[q]] = acc;
  }
}

__device__ __forceinline__ bool fused_sums(const RepInfo& R, int apb) {
  return (R.ipad_end - R.ioff) / apb <= kFusedBlocks;
}

// Thermostat on the full-step velocities, then (unless last) the next
// half-kick and drift.
// The kinetic energy comes from the force launch's partials (summed here
// for replicas of at most kFusedBlocks force blocks of apb atoms, else from
// the reduction launch).  All 64 lanes of a wave call it together.
// Contexts of at least this many (padded) atoms bin the thermostat kernel's
// drifted positions with one atomic per distinct cell of a wavefront: the
// replica table (~2.8e5 atoms, throughput bound) gains 3.5 us per step, a
// 4096-atom box (latency bound) would lose ~3 us per launch to the extra pass.
constexpr long long kAggAtoms = 65536;

__device__ __forceinline__ void thermostat_atom(const Dev& d, const Phys& p, int par, int last, int i, int apb,
                                                unsigned tid) {
  const bool agg = d.npad >= kAggAtoms;
  if (i < d.npad) {
    // the atom's records before the replica lookup (padded arrays), pinned
    // so their round trip overlaps it
    const float4 vi = d.v[i], Fi = d.f[i];
    const uint4 ui = pick(d.u, par)[i], urefi = d.uref[i];
    const int rep = d.R == 1 ? 0 : __builtin_amdgcn_readfirstlane(d.tile_rep[i >> 6]);
    asm volatile("" ::"v"(vi.x), "v"(Fi.x), "v"(ui.x), "v"(urefi.x));
    const RepInfo& R = d.reps[rep];
    int bc = -1;
    uint4 be = make_uint4(0u, 0u, 0u, 0u);
    double ke;
    if (fused_sums(R, apb)) {
      const int ks[4] = {2, 2, 2, 2};
      double th[kNQ];
      replica_sums(d, apb, R, ks, 1, th, tid);
      ke = th[2];
    } else {
      ke = d.thermo_cur[rep * kNQ + 2];
    }
    if (i < R.iend) {
      const double T = 2.0 * ke / R.ndof_kb;
      const double T0 = d.T0[rep];
      double s = 1.0;
      if (T > 0.0) {
        s = p.thermostat == 1 ? sqrt(T0 / T) : sqrt(fmax(0.0, 1.0 + p.dt_d / p.tau_d * (T0 / T - 1.0)));
      }
      float4 v = vi;
      const float sf = (float)s;
      v.x *= sf; v.y *= sf; v.z *= sf;
      if (!last) {
        v.x += p.hdt_cm * Fi.x; v.y += p.hdt_cm * Fi.y; v.z += p.hdt_cm * Fi.z;
        uint4 un = ui;
        const int c = drift(d, geo_of(R), rep, i, un, v, urefi, p.dt, p.half_skin, par ^ 1);
        const uint4 e = make_uint4(un.x, un.y, un.z, (unsigned)i);
        if (agg) {
          bc = c;
          be = e;
        } else {
          cell_put(d, par ^ 1, c, e);
        }
      }
      d.v[i] = v;
    }
    if (!last && agg) cell_append(d, par ^ 1, bc, be);   // npad is a multiple of 64: whole wavefronts
  }
}

__global__ __launch_bounds__(kBlock) void k_thermostat(Dev d, Phys p, int par, int last, int apb) {
  thermostat_atom(d, p, par, last, blockIdx.x * kBlock + threadIdx.x, apb, threadIdx.x);
}

// ----------------------------------------------------------------- isobaric
// Nose-Hoover chains and the isotropic barostat (the thermostat and barostat
// of Sec. II.B, read as the Martyna-Tobias-Klein equations; one step of
// length dt = 2h is the symmetric splitting
//   chain(eta) chain(xi) baro kick(h) drift(dt) kick(h) baro chain(xi) chain(eta)).
// One launch closes the previous step (baro, particle chain, barostat chain,
// record) and opens the next one (barostat chain, particle chain, baro,
// first kick, drift with the box scaling, binning); the force launch makes
// the second kick.  The per-replica arithmetic is FP64 and repeated by every
// thread of the replica (identical inputs, identical results); the thread
// of the replica's first atom stores the new state, box and kick
// coefficients.

// exp and sinh(x)/x for the small arguments of the chain and box factors
// (|x| of order h / tau): Taylor series by Horner's rule for |x| <= 1/16,
// where the first omitted term is below 2^-60 relative (x^10 / 10! and
// x^10 / 11!), else the library functions.  The chain is a serial run of
// such factors, so a short dependent series is the step's critical path.
__device__ __forceinline__ double exp_small(double x) {
  if (fabs(x) > 0.0625) return exp(x);
  double r = 1.0 / 362880.0;                                  // 1/9!
  r = fma(r, x, 1.0 / 40320.0);
  r = fma(r, x, 1.0 / 5040.0);
  r = fma(r, x, 1.0 / 720.0);
  r = fma(r, x, 1.0 / 120.0);
  r = fma(r, x, 1.0 / 24.0);
  r = fma(r, x, 1.0 / 6.0);
  r = fma(r, x, 0.5);
  r = fma(r, x, 1.0);
  return fma(r, x, 1.0);
}

__device__ __forceinline__ double sinhc_d(double x) {
  if (fabs(x) > 0.0625) return sinh(x) / x;
  const double y = x * x;
  double r = 1.0 / 362880.0;                                  // 1/9!
  r = fma(r, y, 1.0 / 5040.0);
  r = fma(r, y, 1.0 / 120.0);
  r = fma(r, y, 1.0 / 6.0);
  return fma(r, y, 1.0);
}

// One chain half step of length h on a subsystem with kinetic term k2 (twice
// its kinetic energy) and nf degrees of freedom; returns the velocity scale.
// Q / iQ are the link masses and reciprocals; the chain length M is a
// template argument, so every index is a constant, the chain stays in
// registers, and the particle and barostat chains (independent within a
// half step) form one straight-line block the scheduler can interleave.
template <int M>
__device__ __forceinline__ double chain_half(double h, double& k2, double nfkT, double kT, const double* Q,
                                             const double* iQ, double* x, double* vx) {
  auto g = [&](int k) { return k == 0 ? (k2 - nfkT) * iQ[0] : (Q[k - 1] * vx[k - 1] * vx[k - 1] - kT) * iQ[k]; };
#pragma unroll
  for (int k = kNptChain - 1; k >= 0; --k) {
    if (k == M - 1) {
      vx[k] += 0.5 * h * g(k);
    } else if (k < M - 1) {
      const double e = exp_small(-0.25 * h * vx[k + 1]);
      vx[k] = (vx[k] * e + 0.5 * h * g(k)) * e;
    }
  }
  const double sc = exp_small(-h * vx[0]);
  k2 *= sc * sc;
#pragma unroll
  for (int k = 0; k < kNptChain; ++k)
    if (k < M) x[k] += h * vx[k];
#pragma unroll
  for (int k = 0; k < kNptChain; ++k) {
    if (k < M - 1) {
      const double e = exp_small(-0.25 * h * vx[k + 1]);
      vx[k] = (vx[k] * e + 0.5 * h * g(k)) * e;
    } else if (k == M - 1) {
      vx[k] += 0.5 * h * g(k);
    }
  }
  return sc;
}

template <int M, bool BARO>
__global__ __launch_bounds__(kBlock) void k_npt_kick(Dev d, Phys p, NptArgs a) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= d.npad) return;
  // The atom's records are loaded before the replica is known (the arrays
  // are padded to npad, so the padding lanes read in bounds) and pinned
  // here, so their round trip overlaps the replica lookup instead of
  // following the chain arithmetic.
  const float4 vi = d.v[i], Fi = d.f[i];
  const uint4 ui = pick(d.u, a.par)[i], urefi = d.uref[i];
  // one wave is one tile of one replica: the replica's records load as scalars
  const int rep = d.R == 1 ? 0 : __builtin_amdgcn_readfirstlane(d.tile_rep[i >> 6]);
  asm volatile("" ::"v"(vi.x), "v"(Fi.x), "v"(ui.x), "v"(urefi.x));
  const RepInfo& R = d.reps[rep];
  NptState st = a.in[rep];
  const NptConst C = a.cst[rep];
  const double h = 0.5 * a.dt;
  const double nfkT = C.nf * C.kT;
  const double Qb[kNptChain] = {C.Qb, C.Qb, C.Qb, C.Qb};
  const double iQb[kNptChain] = {C.iQb, C.iQb, C.iQb, C.iQb};
  static_assert(kNptChain == 4, "barostat chain constants are spelled out for four links");
  constexpr bool baro = BARO;                // no barostat: fixed box (NVT)
  double th[kNQ];
  const bool rec_wave = a.row && (a.mode & NPT_END) && (i >> 6) == (R.ioff >> 6);
  if (fused_sums(R, a.apb)) {
    // The step needs the kinetic and virial sums (2..5); the wave that
    // writes a record also sums the energies and the tensor diagonal.  The
    // choice of in-kernel sums depends on the replica alone, so a replica's
    // arithmetic is the same whatever shares its context.
#pragma unroll
    for (int k = 0; k < kNQ; ++k) th[k] = 0.0;
    const int kin[4] = {2, 3, 4, 5}, rec1[4] = {0, 1, 9, 10}, rec2[4] = {11, 11, 11, 11};
    replica_sums(d, a.apb, R, kin, 4, th, threadIdx.x);
    if (rec_wave) {
      replica_sums(d, a.apb, R, rec1, 4, th, threadIdx.x);
      replica_sums(d, a.apb, R, rec2, 1, th, threadIdx.x);
    }
  } else {
#pragma unroll
    for (int k = 0; k < kNQ; ++k) th[k] = d.thermo_cur[(size_t)rep * kNQ + k];
  }
  const double W = th[3] + th[4] + th[5];
  double k2 = 2.0 * th[2];
  double vs = 1.0;
  const bool lead = i == R.ioff;
  if (a.mode & NPT_END) {
    const double V = st.L[0] * st.L[1] * st.L[2];
    if (baro) st.ve += h * (C.alpha * k2 + W - 3.0 * C.pext * V) * C.iWb;
    vs = chain_half<M>(h, k2, nfkT, C.kT, C.Q, C.iQ, st.xi, st.vxi);
    if (baro) {
      double kb2 = C.Wb * st.ve * st.ve;
      st.ve *= chain_half<M>(h, kb2, C.kT, C.kT, Qb, iQb, st.eta, st.veta);
    }
    if (lead && a.row) {
      double ext = baro ? 0.5 * C.Wb * st.ve * st.ve : 0.0;
#pragma unroll
      for (int k = 0; k < kNptChain; ++k) {
        if (k >= M) continue;
        ext += 0.5 * C.Q[k] * st.vxi[k] * st.vxi[k] + (k == 0 ? C.nf : 1.0) * C.kT * st.xi[k];
        if (baro) ext += 0.5 * C.Qb * st.veta[k] * st.veta[k] + C.kT * st.eta[k];
      }
      const double U = th[0] + th[1], ke = 0.5 * k2, v2 = vs * vs;
      double* row = a.row + (size_t)rep * kNptRow;
      row[0] = V; row[1] = (k2 + W) / (3.0 * V) / kBar; row[2] = k2 / (C.nf * kBoltz); row[3] = U;
      row[4] = ke; row[5] = C.pext * V; row[6] = ext; row[7] = ke + U + C.pext * V + ext;
      for (int c = 0; c < 3; ++c) row[8 + c] = (v2 * th[9 + c] + th[3 + c]) / V / kBar;   // P_aa
    }
  }
  float ka = 1.f, kb = 0.f, tx = 0.f, hs = 0.f;
  Geo G{};
  if (a.mode & NPT_BEGIN) {
    if (baro) {
      double kb2 = C.Wb * st.ve * st.ve;
      st.ve *= chain_half<M>(h, kb2, C.kT, C.kT, Qb, iQb, st.eta, st.veta);
    }
    vs *= chain_half<M>(h, k2, nfkT, C.kT, C.Q, C.iQ, st.xi, st.vxi);
    const double V = st.L[0] * st.L[1] * st.L[2];
    if (baro) st.ve += h * (C.alpha * k2 + W - 3.0 * C.pext * V) * C.iWb;
    const double c = C.alpha * st.ve;
    ka = (float)exp_small(-c * h);
    kb = (float)(h * a.c_m * exp_small(-0.5 * c * h) * sinhc_d(0.5 * c * h));
    const double gr = exp_small(st.ve * a.dt);
    tx = (float)(a.dt * exp_small(0.5 * st.ve * a.dt) * sinhc_d(0.5 * st.ve * a.dt));
    for (int k = 0; k < 3; ++k) st.L[k] *= gr;
    hs = (float)(0.5 * (st.L[0] / d.lref[rep] * a.rl - a.rc) - 1e-4);
    G = Geo{(float)(st.L[0] / kTwo32), (float)(st.L[1] / kTwo32), (float)(st.L[2] / kTwo32),
            (float)(kTwo32 / st.L[0]), (float)(kTwo32 / st.L[1]), (float)(kTwo32 / st.L[2]),
            R.nc[0], R.nc[1], R.nc[2], R.cell_off};
  }
  if (i < R.iend) {
    float4 v = vi;
    const float fs = (float)vs;
    v.x *= fs; v.y *= fs; v.z *= fs;
    if (a.mode & NPT_BEGIN) {
      v.x = ka * v.x + kb * Fi.x; v.y = ka * v.y + kb * Fi.y; v.z = ka * v.z + kb * Fi.z;
      uint4 un = ui;
      const int c = drift(d, G, rep, i, un, v, urefi, tx, hs, a.par ^ 1);
      cell_put(d, a.par ^ 1, c, make_uint4(un.x, un.y, un.z, (unsigned)i));
    }
    d.v[i] = v;
  }
  if (lead) {
    a.out[rep] = st;
    if (a.mode & NPT_BEGIN) {
      a.kick[rep] = make_float2(ka, kb);
      RepInfo& Rw = a.reps[rep];
      for (int k = 0; k < 3; ++k) {
        Rw.L[k] = st.L[k];
        Rw.scale[k] = (float)(st.L[k] / kTwo32);
        Rw.inv_scale[k] = (float)(kTwo32 / st.L[k]);
        if (st.L[k] / R.nc[k] < a.rl) atomicOr(&d.flags[F_BOX], 1);
      }
    }
  }
}

// ----------------------------------------------------------------- persistent
// Waits of a persistent launch.  Every wait is bounded: a block that waits
// too long raises `abort`, and every later wait returns at once, so the
// grid always drains.  Counters are read at agent scope (past the L1).
__device__ bool wait_count(const PArgs& a, unsigned* w, unsigned target, unsigned mask, unsigned* seen) {
  unsigned spins = 0;
  for (;;) {
    const unsigned v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((v & mask) >= target) {
      *seen = v;
      return true;
    }
    if (__hip_atomic_load(a.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    __builtin_amdgcn_s_sleep(2);
    if (++spins > (1u << 22)) {
      atomicOr(a.abort, 1);
      return false;
    }
  }
}

// Grid-wide barrier: arrivals add to a counter that only grows (barrier k
// completes at k * G arrivals).  Blocks on different XCCs exchange data
// through it, and each XCC has its own L2, so every block writes back and
// invalidates its XCC's L2 (agent-scope release and acquire).
__device__ bool grid_sync(const PArgs& a, unsigned G, unsigned& k) {
  __shared__ int ok;
  __builtin_amdgcn_s_waitcnt(0);           // this wave's stores have reached the L2
  __syncthreads();
  ++k;
  if (threadIdx.x == 0) {
    __threadfence();                       // release this block's writes
    atomicAdd(a.ctl + kCtlGrid, 1u);
    unsigned v;
    const bool good = wait_count(a, a.ctl + kCtlGrid, k * G, ~0u, &v);
    __threadfence();                       // acquire the other blocks' writes
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

// After group barrier k: drops the compute unit's L1 lines once.  The
// first block of the CU past the barrier invalidates (an agent-scope
// acquire: on this chip a narrower invalidate leaves the L1 lines in
// place) and marks k done; the CU's other blocks wait for the mark.  An
// invalidate costs each XCC's L2 tens of nanoseconds in turn, so one per
// CU rather than per block shortens every barrier.
__device__ bool drop_l1(const PArgs& a, unsigned* cu, unsigned k) {
  if (atomicMax(cu + kCtlEpoch, k) < k) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __builtin_amdgcn_s_waitcnt(0);
    atomicMax(cu + kCtlDone, k);
    return true;
  }
  unsigned v;
  return wait_count(a, cu + kCtlDone, k, ~0u, &v);
}

// Barrier of the blocks on one XCC (group form).  A replica's data is only
// touched by its group, and a group's writes all land in its XCC's L2, so
// nothing is written back; only the L1 lines go (drop_l1).  Barrier k of
// the group completes at k * nb arrivals (nb blocks in the group); `cu` is
// a.ctl offset by the block's CU (256 x + cu_key()).
__device__ bool group_sync(const PArgs& a, unsigned* ctr, unsigned k, unsigned nb, unsigned* cu) {
  __shared__ int ok;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(ctr, 1u);
    unsigned v;
    ok = wait_count(a, ctr, k * nb, ~0u, &v) && drop_l1(a, cu, k);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  return ok != 0;
}

// End of a step in the group form with synchronised rebuilds: the group's
// last block to arrive ORs the rebuild flags its blocks raised for the
// next step (parity npar) and adds one arrival, with the flag, to the
// step's word; every block waits until all groups have added theirs, which
// also completes its own group's barrier.  `any` becomes the OR over all
// replicas, as the one-launch-per-phase form reads it.
__device__ bool step_sync(const PArgs& a, const Dev& d, unsigned* ctr, unsigned k, unsigned nb, unsigned* cu,
                          unsigned* word, const int* reps, int rlo, int rhi, int npar, int& any) {
  __shared__ int ok, fl;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned old = atomicAdd(ctr, 1u);
    if (old + 1u == k * nb) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      int f = 0;
      for (int j = rlo; j < rhi; ++j) f |= d.dflag[npar * d.R + reps[j]];
      atomicAdd(word, 1u | (f != 0 ? 256u : 0u));
    }
    unsigned v = 0;
    ok = wait_count(a, word, (unsigned)a.ng, 0xffu, &v) && drop_l1(a, cu, k);
    fl = (v >> 8) != 0u;
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  any = fl;
  return ok != 0;
}

// Maps the group-relative units (tiles of `unit` atoms) of the group's
// replicas, taken in table order and visited in increasing order, to
// global unit numbers.
struct GroupCursor {
  int j, acc, n, first;
  __device__ __forceinline__ int at(const Dev& d, const int* reps, int unit, int k) {
    while (k >= acc + n) {
      acc += n;
      const RepInfo& R = d.reps[reps[j++]];
      first = R.ioff / unit;
      n = (R.ipad_end - R.ioff) / unit;
    }
    return first + k - acc;
  }
};

// Clears, for the group's replicas, what clear_next clears for all.
__device__ __forceinline__ void clear_group(const Dev& d, int par, const int* reps, int rlo, int rhi, unsigned slot,
                                            unsigned nb, unsigned tid) {
  for (int j = rlo; j < rhi; ++j) {
    const int r = reps[j];
    const RepInfo& R = d.reps[r];
    if (slot == 0 && tid == 0) d.dflag[(par ^ 1) * d.R + r] = 0;
    for (int c = (int)(slot * kBlock + tid); c < R.ncell; c += (int)(nb * kBlock)) pick(d.gcnt, par ^ 1)[R.cell_off + c] = 0;
  }
}

// All steps t0..t1 of sw_step in one launch: the same tile functions as the
// one-kernel-per-phase path, separated by barriers.
//   Grid form (ng = 1): worker w (blocks remapped per XCC) owns a
//   contiguous range of tiles in every phase; grid-wide barriers.
//   Group form (ng > 1): the replicas are dealt to the XCCs (the group
//   table); the blocks found on an XCC share its replicas' tiles and
//   synchronise among themselves, so no barrier writes back an L2.  With
//   synchronised rebuilds the groups also meet once per step, through one
//   word per step.  A census at the start checks that blocks run on exactly
//   the XCCs the table names; otherwise the launch takes the grid form.
// Both forms give the same bits as one launch per phase: every tile's
// arithmetic is independent of which block runs it.
// Four wavefronts per SIMD (128 VGPRs): the loop over steps holds state
// that one launch per phase does not, and without the bound the kernel
// takes 133 VGPRs and three wavefronts (no spills at 8 or more lanes per
// atom; five wavefronts would spill 52 VGPRs).
template <int LPA>
__global__ __launch_bounds__(kBlock, 4) void k_persistent(Dev d, Phys p, PArgs a) {
  constexpr int APB = kBlock / LPA;
  extern __shared__ int lds[];
  __shared__ unsigned sh_census[3];
  const unsigned G = gridDim.x;
  unsigned kgrid = 0;
  const unsigned xc = xcc_id();
  bool grouped = false;
  unsigned slot = (unsigned)xcd_remap(blockIdx.x, (int)G), nb = G;
  if (a.ng > 1) {
    if (threadIdx.x == 0) sh_census[0] = atomicAdd(a.ctl + kCtlCensus + xc, 1u);
    if (!grid_sync(a, G, kgrid)) return;
    if (threadIdx.x == 0) {
      unsigned good = (a.xmask >> xc) & 1u;
      for (int x = 0; x < kMaxXcc; ++x) {
        const unsigned c = __hip_atomic_load(a.ctl + kCtlCensus + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((c != 0u) != (((a.xmask >> x) & 1u) != 0u)) good = 0u;
        if (x == (int)xc) sh_census[1] = c;
      }
      sh_census[2] = good;
    }
    __syncthreads();
    if (sh_census[2] != 0u) {
      grouped = true;
      slot = sh_census[0];
      nb = sh_census[1];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicMax(&d.flags[F_PGROUPS], grouped ? a.ng : 1);
  // the block's share of tiles and 64-atom waves (group form: numbered
  // within the group), and the group's replicas
  const int* reps = nullptr;
  long long nt = d.npad / APB, nw = d.npad / kTile;
  int rlo = 0, rhi = 0;
  if (grouped) {
    const int ng = a.ng;
    const int g = __builtin_popcount(a.xmask & ((1u << xc) - 1u));
    const int* woff = a.gtab;
    const int* roff = woff + (ng + 1);
    reps = roff + (ng + 1);
    nw = woff[g + 1] - woff[g];
    nt = nw * (kTile / APB);
    rlo = roff[g];
    rhi = roff[g + 1];
  }
  const int tlo = (int)(nt * slot / nb), thi = (int)(nt * (slot + 1) / nb);
  const int wlo = (int)(nw * slot / nb), whi = (int)(nw * (slot + 1) / nb);
  unsigned* gctr = a.ctl + kCtlGroup + 64 * xc;
  unsigned* cu = a.ctl + 256 * xc + cu_key();
  unsigned kgrp = 0;
  // Synchronised rebuilds (a.sync_rb; d.sync_rb is 0 here, so a tile reads
  // only its own replica's flag): `any` is the OR of every replica's flag
  // for the coming step, taken by each block from the flags themselves
  // where they are visible to it (the first step, whose flags were written
  // before the launch, and every step of the grid form, after its
  // grid-wide barrier) and from the step words in the group form.
  int any = 0;
  auto all_flags = [&](int par) {
    int f = 0;
    for (int r = 0; r < d.R; ++r) f |= d.dflag[par * d.R + r];
    return f != 0 ? 1 : 0;
  };
  const bool thermostat = p.thermostat != 0;
  auto sync = [&]() -> bool { return grouped ? group_sync(a, gctr, ++kgrp, nb, cu) : grid_sync(a, G, kgrid); };
  auto sync_end = [&](int t) -> bool {
    if (!(grouped && a.sync_rb)) return sync();
    return step_sync(a, d, gctr, ++kgrp, nb, cu, a.ctl + kCtlStep + (t - a.t0), reps, rlo, rhi, (t + 1) & 1, any);
  };
  for (int t = a.t0; t <= a.t1; ++t) {
    const int par = t & 1;
    if (a.sync_rb && (t == a.t0 || !grouped)) any = all_flags(par);
    const bool rec = a.thermo_every > 0 && t % a.thermo_every == 0;
    const bool last = t == a.nsteps;
    const int frb = (a.rebuild_every > 0 && t % a.rebuild_every == 0) || any;
    double* row = rec && a.thermo ? a.thermo + (size_t)(t / a.thermo_every - 1) * d.R * kNQ : nullptr;
    GroupCursor cm{rlo, 0, 0, 0};
    for (int k = tlo; k < thi; ++k) {
      const int b = grouped ? cm.at(d, reps, APB, k) : k;
      if (rec) moments_tile<LPA, true>(d, p, par, frb, b, opaque_tid(), lds);
      else moments_tile<LPA, false>(d, p, par, frb, b, opaque_tid(), lds);
    }
    if (grouped) clear_group(d, par, reps, rlo, rhi, slot, nb, opaque_tid());
    else clear_next(d, par, blockIdx.x, (int)G, opaque_tid());
    if (!sync()) return;
    GroupCursor cf{rlo, 0, 0, 0};
    for (int k = tlo; k < thi; ++k) {
      const int b = grouped ? cf.at(d, reps, APB, k) : k;
      if (thermostat) {
        if (rec) forces_tile<LPA, MODE_KICK, true>(d, p, par, b, opaque_tid());
        else forces_tile<LPA, MODE_KICK, false>(d, p, par, b, opaque_tid());
      } else if (last) {
        if (rec) forces_tile<LPA, MODE_NVE_LAST, true>(d, p, par, b, opaque_tid());
        else forces_tile<LPA, MODE_NVE_LAST, false>(d, p, par, b, opaque_tid());
      } else {
        if (rec) forces_tile<LPA, MODE_NVE, true>(d, p, par, b, opaque_tid());
        else forces_tile<LPA, MODE_NVE, false>(d, p, par, b, opaque_tid());
      }
    }
    // per-replica sums of the force phase's partials: for thermo rows, and
    // for a thermostat on replicas too large for the thermostat phase to
    // sum itself (as the per-phase launches)
    if (rec || (thermostat && needs_reduce_launch(d, APB))) {
      if (!sync()) return;
      if (grouped) {
        const int ntask = (rhi - rlo) * kNQ;
        for (int j = (int)slot; j < ntask; j += (int)nb)
          reduce_task(d, APB, row, reps[rlo + j / kNQ] * kNQ + j % kNQ, opaque_tid());
      } else {
        for (int task = (int)slot; task < d.R * kNQ; task += (int)G) reduce_task(d, APB, row, task, opaque_tid());
      }
    }
    if (!thermostat) {
      if (!sync_end(t)) return;
      continue;
    }
    if (!sync()) return;
    // the block's waves take its 64-atom units in turn
    GroupCursor ct{rlo, 0, 0, 0};
    for (int k = wlo + (int)(threadIdx.x >> 6); k < whi; k += kBlock / 64) {
      const int u = grouped ? ct.at(d, reps, kTile, k) : k;
      const unsigned tid = opaque_tid();
      thermostat_atom(d, p, par, last, u * kTile + (int)(tid & 63), APB, tid);
    }
    if (!sync_end(t)) return;
  }
}

__global__ __launch_bounds__(kBlock) void k_scatter_out(Dev d, int par, float4* __restrict__ x,
                                                       float4* __restrict__ v, float4* __restrict__ f) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= d.npad) return;
  const int k = d.ids[i];
  if (k < 0) return;
  const RepInfo& R = d.reps[d.tile_rep[i >> 6]];
  if (x) {
    const uint4 u = d.u[par][i];
    x[k] = make_float4((float)((double)u.x * (R.L[0] / kTwo32)), (float)((double)u.y * (R.L[1] / kTwo32)),
                       (float)((double)u.z * (R.L[2] / kTwo32)), 0.f);
  }
  if (v) {
    float4 a = d.v[i];
    a.w = 0.f;
    v[k] = a;
  }
  if (f) {
    float4 a = d.f[i];
    a.w = 0.f;
    f[k] = a;
  }
}

__global__ void k_copy_thermo(const double* __restrict__ cur, int R, double* energy, double* virial) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  if (energy) {
    energy[2 * r] = cur[r * kNQ + 0];
    energy[2 * r + 1] = cur[r * kNQ + 1];
  }
  if (virial)
    for (int k = 0; k < 6; ++k) virial[6 * r + k] = cur[r * kNQ + 3 + k];
}

__global__ void k_fill_i32(int* p, int value, long long n) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = value;
}
__global__ void k_fill_f32(float* p, float value, long long n) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = value;
}

__global__ void k_fill_f64(double* p, double value, long long n) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = value;
}

inline unsigned nblk(long long n, int b) { return (unsigned)((n + b - 1) / b); }

// Launches go through hipExtLaunchKernelGGL so that sampled launches can
// carry start/stop events recorded at the dispatch itself.
template <int LPA>
hipError_t moments_lpa(const Dev& d, const Phys& p, int par, int force_rebuild, int energy, hipStream_t s,
                       const KTimer& tm) {
  constexpr int APB = kBlock / LPA;
  const uint32_t lds = (uint32_t)moments_lds_bytes(APB, d.cap);
  const unsigned grid = (unsigned)(d.npad / APB);
  if (!tm.start && !tm.stop) {   // plain launch (also the form used under graph capture)
    if (energy) hipLaunchKernelGGL((k_moments<LPA, true>), dim3(grid), dim3(kBlock), lds, s, d, p, par, force_rebuild);
    else hipLaunchKernelGGL((k_moments<LPA, false>), dim3(grid), dim3(kBlock), lds, s, d, p, par, force_rebuild);
  } else if (energy) {
    hipExtLaunchKernelGGL((k_moments<LPA, true>), dim3(grid), dim3(kBlock), lds, s, tm.start, tm.stop, 0u, d, p,
                          par, force_rebuild);
  } else {
    hipExtLaunchKernelGGL((k_moments<LPA, false>), dim3(grid), dim3(kBlock), lds, s, tm.start, tm.stop, 0u, d, p,
                          par, force_rebuild);
  }
  return hipGetLastError();
}

template <int LPA, int MODE>
hipError_t forces_mode(const Dev& d, const Phys& p, int vir, int par, double* ring_row, hipStream_t s,
                       const KTimer& tm, bool reduce = true) {
  constexpr int APB = kBlock / LPA;
  const unsigned grid = (unsigned)(d.npad / APB);
  if (!tm.start && !tm.stop) {
    if (vir) hipLaunchKernelGGL((k_forces<LPA, MODE, true>), dim3(grid), dim3(kBlock), 0, s, d, p, par);
    else hipLaunchKernelGGL((k_forces<LPA, MODE, false>), dim3(grid), dim3(kBlock), 0, s, d, p, par);
  } else if (vir) {
    hipExtLaunchKernelGGL((k_forces<LPA, MODE, true>), dim3(grid), dim3(kBlock), 0u, s, tm.start, tm.stop, 0u, d, p,
                          par);
  } else {
    hipExtLaunchKernelGGL((k_forces<LPA, MODE, false>), dim3(grid), dim3(kBlock), 0u, s, tm.start, tm.stop, 0u, d,
                          p, par);
  }
  // the kick is followed by the thermostat launch, which sums small replicas itself
  if (reduce && (vir || (MODE == MODE_KICK && needs_reduce_launch(d, APB))))
    hipLaunchKernelGGL(k_reduce_thermo, dim3((unsigned)min(d.R * kNQ, 4096)), dim3(kBlock), 0, s, d, APB, ring_row);
  return hipGetLastError();
}

template <int LPA>
hipError_t forces_lpa(const Dev& d, const Phys& p, int mode, int vir, int par, double* ring_row, hipStream_t s,
                      const KTimer& tm) {
  switch (mode) {
    case MODE_FORCES: return forces_mode<LPA, MODE_FORCES>(d, p, 1, par, ring_row, s, tm);
    case MODE_START: return forces_mode<LPA, MODE_START>(d, p, vir, par, ring_row, s, tm);
    case MODE_NVE: return forces_mode<LPA, MODE_NVE>(d, p, vir, par, ring_row, s, tm);
    case MODE_NVE_LAST: return forces_mode<LPA, MODE_NVE_LAST>(d, p, vir, par, ring_row, s, tm);
    case MODE_KICK: return forces_mode<LPA, MODE_KICK>(d, p, vir, par, ring_row, s, tm);
    // isobaric: sums always; vir = 0 leaves the block partials to the kick launch
    case MODE_NPT: return forces_mode<LPA, MODE_NPT>(d, p, 1, par, ring_row, s, tm, vir != 0);
  }
  return hipErrorInvalidValue;
}

__global__ void k_xcc_census(unsigned* word) {
  if (threadIdx.x == 0) atomicOr(word, 1u << xcc_id());
}

template <int LPA>
hipError_t persistent_lpa(const Dev& d, const Phys& p, const PArgs& a, int blocks_per_cu, hipStream_t s,
                          int* grid_out) {
  constexpr int APB = kBlock / LPA;
  const size_t lds = moments_lds_bytes(APB, d.cap);
  int per_cu = 0, dev = 0, ncu = 0;
  hipError_t e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<LPA>, kBlock, lds)) != hipSuccess)
    return e;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  if (blocks_per_cu > 0) per_cu = min(per_cu, blocks_per_cu);
  const int ntile = d.npad / APB;
  const int grid = max(1, min(per_cu * ncu, ntile));
  *grid_out = grid;
  Dev dd = d;
  dd.sync_rb = 0;           // the kernel takes synchronised rebuilds from PArgs
  Phys pp = p;
  PArgs aa = a;
  aa.sync_rb = d.sync_rb;
  void* args[] = {&dd, &pp, &aa};
  return hipLaunchCooperativeKernel((const void*)k_persistent<LPA>, dim3(grid), dim3(kBlock), args,
                                    (unsigned)lds, s);
}

}  // namespace

hipError_t xcc_census(unsigned* d_word, unsigned* mask_out, hipStream_t s) {
  hipError_t e;
  int dev = 0, ncu = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  if ((e = launch_fill_i32((int*)d_word, 0, 1, s)) != hipSuccess) return e;
  // a few blocks per compute unit: the dispatcher deals them to every XCC
  hipLaunchKernelGGL(k_xcc_census, dim3(4 * max(ncu, 1)), dim3(64), 0, s, d_word);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  unsigned h = 0;
  if ((e = hipMemcpyAsync(&h, d_word, sizeof h, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  *mask_out = h;
  return hipSuccess;
}

hipError_t launch_persistent(const Dev& d, const Phys& p, int lpa, const PArgs& a, int blocks_per_cu,
                             hipStream_t s, int* grid_out) {
  hipError_t e;
  if ((e = launch_fill_i32((int*)a.ctl, 0, kCtlWords, s)) != hipSuccess) return e;
  switch (lpa) {
    case 4: return persistent_lpa<4>(d, p, a, blocks_per_cu, s, grid_out);
    case 8: return persistent_lpa<8>(d, p, a, blocks_per_cu, s, grid_out);
    case 16: return persistent_lpa<16>(d, p, a, blocks_per_cu, s, grid_out);
    case 32: return persistent_lpa<32>(d, p, a, blocks_per_cu, s, grid_out);
    case 64: return persistent_lpa<64>(d, p, a, blocks_per_cu, s, grid_out);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sort(const Dev& d, const float4* x_user, const float4* v_user, long long n_user,
                       const long long* uoff, int R, const int* cell_rank, uint4* uq, int* key, int* cnt,
                       int* start, int* cursor, int* order, hipStream_t s) {
  hipError_t e;
  if ((e = launch_fill_i32(cnt, 0, d.ctot, s)) != hipSuccess) return e;
  if ((e = launch_fill_i32(cursor, 0, d.ctot, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_sort_count, dim3(nblk(n_user, kBlock)), dim3(kBlock), 0, s, x_user, n_user, uoff, R,
                     d.reps, cell_rank, uq, key, cnt);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, cnt, start, d.ctot);
  hipLaunchKernelGGL(k_sort_scatter, dim3(nblk(n_user, kBlock)), dim3(kBlock), 0, s, n_user, key, start, cursor,
                     order);
  hipLaunchKernelGGL(k_sort_cells, dim3(nblk(d.ctot, kBlock)), dim3(kBlock), 0, s, d.ctot, cnt, start, order);
  hipLaunchKernelGGL(k_gather_sorted, dim3(nblk(d.npad, kBlock)), dim3(kBlock), 0, s, d, uq, v_user, order);
  return hipGetLastError();
}

hipError_t launch_gather_ids(const Dev& d, const float4* x_user, int par, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_ids, dim3(nblk(d.npad, kBlock)), dim3(kBlock), 0, s, d, x_user, par);
  return hipGetLastError();
}

hipError_t launch_bin(const Dev& d, int par, int check_disp, float rl, float rc, hipStream_t s) {
  hipLaunchKernelGGL(k_bin, dim3(nblk(d.npad, kBlock)), dim3(kBlock), 0, s, d, par, check_disp, rl, rc);
  return hipGetLastError();
}

hipError_t launch_moments(const Dev& d, const Phys& p, int lpa, int par, int force_rebuild, int energy,
                          hipStream_t s, const KTimer& tm) {
  switch (lpa) {
    case 4: return moments_lpa<4>(d, p, par, force_rebuild, energy, s, tm);
    case 8: return moments_lpa<8>(d, p, par, force_rebuild, energy, s, tm);
    case 16: return moments_lpa<16>(d, p, par, force_rebuild, energy, s, tm);
    case 32: return moments_lpa<32>(d, p, par, force_rebuild, energy, s, tm);
    case 64: return moments_lpa<64>(d, p, par, force_rebuild, energy, s, tm);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_moments_tan(const Dev& d, const Phys& p, int lpa, int par, int force_rebuild, const float4* w,
                              float4* mdot, hipStream_t s) {
  const unsigned grid = (unsigned)(d.npad / (kBlock / lpa));
  const uint32_t lds = (uint32_t)moments_lds_bytes(kBlock / lpa, d.cap);
  switch (lpa) {
    case 4: hipLaunchKernelGGL(k_moments_tan<4>, dim3(grid), dim3(kBlock), lds, s, d, p, par, force_rebuild, w, mdot); break;
    case 8: hipLaunchKernelGGL(k_moments_tan<8>, dim3(grid), dim3(kBlock), lds, s, d, p, par, force_rebuild, w, mdot); break;
    case 16: hipLaunchKernelGGL(k_moments_tan<16>, dim3(grid), dim3(kBlock), lds, s, d, p, par, force_rebuild, w, mdot); break;
    case 32: hipLaunchKernelGGL(k_moments_tan<32>, dim3(grid), dim3(kBlock), lds, s, d, p, par, force_rebuild, w, mdot); break;
    case 64: hipLaunchKernelGGL(k_moments_tan<64>, dim3(grid), dim3(kBlock), lds, s, d, p, par, force_rebuild, w, mdot); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_forces(const Dev& d, const Phys& p, int lpa, int mode, int vir, int par, double* ring_row,
                         hipStream_t s, const KTimer& tm) {
  switch (lpa) {
    case 4: return forces_lpa<4>(d, p, mode, vir, par, ring_row, s, tm);
    case 8: return forces_lpa<8>(d, p, mode, vir, par, ring_row, s, tm);
    case 16: return forces_lpa<16>(d, p, mode, vir, par, ring_row, s, tm);
    case 32: return forces_lpa<32>(d, p, mode, vir, par, ring_row, s, tm);
    case 64: return forces_lpa<64>(d, p, mode, vir, par, ring_row, s, tm);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_thermostat(const Dev& d, const Phys& p, int lpa, int par, int last, hipStream_t s) {
  hipLaunchKernelGGL(k_thermostat, dim3(nblk(d.npad, kBlock)), dim3(kBlock), 0, s, d, p, par, last, kBlock / lpa);
  return hipGetLastError();
}

hipError_t launch_audit(const Dev& d, const Phys& p, int par, unsigned long long* counts, hipStream_t s) {
  hipLaunchKernelGGL(k_audit, dim3(nblk(d.npad, kBlock)), dim3(kBlock), 0, s, d, p, par, counts);
  return hipGetLastError();
}

hipError_t launch_scatter_out(const Dev& d, int par, float4* x_user, float4* v_user, float4* f_user,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_scatter_out, dim3(nblk(d.npad, kBlock)), dim3(kBlock), 0, s, d, par, x_user, v_user,
                     f_user);
  return hipGetLastError();
}

hipError_t launch_copy_thermo(const Dev& d, double* energy, double* virial, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_thermo, dim3(nblk(d.R, 64)), dim3(64), 0, s, d.thermo_cur, d.R, energy, virial);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, int value, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(nblk(n, kBlock)), dim3(kBlock), 0, s, p, value, n);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, float value, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3(nblk(n, kBlock)), dim3(kBlock), 0, s, p, value, n);
  return hipGetLastError();
}

hipError_t launch_npt_kick(const Dev& d, const Phys& p, const NptArgs& a, hipStream_t s) {
  const dim3 grid(nblk(d.npad, kBlock)), block(kBlock);
  static_assert(kNptChain == 4, "one kick instantiation per chain length");
  const bool baro = a.tauP > 0.0;
  switch (a.chain * 2 + (baro ? 1 : 0)) {
    case 2: hipLaunchKernelGGL((k_npt_kick<1, false>), grid, block, 0, s, d, p, a); break;
    case 3: hipLaunchKernelGGL((k_npt_kick<1, true>), grid, block, 0, s, d, p, a); break;
    case 4: hipLaunchKernelGGL((k_npt_kick<2, false>), grid, block, 0, s, d, p, a); break;
    case 5: hipLaunchKernelGGL((k_npt_kick<2, true>), grid, block, 0, s, d, p, a); break;
    case 6: hipLaunchKernelGGL((k_npt_kick<3, false>), grid, block, 0, s, d, p, a); break;
    case 7: hipLaunchKernelGGL((k_npt_kick<3, true>), grid, block, 0, s, d, p, a); break;
    case 8: hipLaunchKernelGGL((k_npt_kick<4, false>), grid, block, 0, s, d, p, a); break;
    case 9: hipLaunchKernelGGL((k_npt_kick<4, true>), grid, block, 0, s, d, p, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, double value, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3(nblk(n, kBlock)), dim3(kBlock), 0, s, p, value, n);
  return hipGetLastError();
}

}  // namespace swk
