// Small device helpers shared by the kernel sources of libsw.
#pragma once
#include "sw_internal.h"

namespace swk {

static __device__ __forceinline__ int xcd_remap(int bid, int G) {
  // Blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous
  // range of (spatially sorted) tiles so neighbour gathers share its L2.
  const int xcd = bid & 7, local = bid >> 3;
  const int per = G >> 3, rem = G & 7;
  return xcd * per + min(xcd, rem) + local;
}

static __device__ __forceinline__ float3 disp(const uint4& a, const uint4& b, const float sc0, const float sc1,
                                       const float sc2) {
  return make_float3((float)(int)(b.x - a.x) * sc0, (float)(int)(b.y - a.y) * sc1,
                     (float)(int)(b.z - a.z) * sc2);
}

static __device__ __forceinline__ int cell_of(const uint4& u, const int nc0, const int nc1, const int nc2) {
  const int cx = (int)__umulhi(u.x, (unsigned)nc0);
  const int cy = (int)__umulhi(u.y, (unsigned)nc1);
  const int cz = (int)__umulhi(u.z, (unsigned)nc2);
  return (cx * nc1 + cy) * nc2 + cz;
}

static __device__ __forceinline__ unsigned quantize(float x, double inv_L) {
  double fr = (double)x * inv_L;
  fr -= floor(fr);
  return (unsigned)(unsigned long long)(fr * kTwo32);  // 2^32 wraps to 0
}

template <int W>
static __device__ __forceinline__ float group_sum(float v) {
#pragma unroll
  for (int m = W / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

static __device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = fmaxf(v, __shfl_xor(v, m, 64));
  return v;
}

// One of the two parity buffers of a device view.  A select of the two
// pointers, not an index: indexing the by-value kernel argument with a
// run-time parity becomes a scalar load that waits for the parity's own
// load, one more round trip at every kernel start.
template <class T>
static __device__ __forceinline__ T pick(T const (&a)[2], int k) {
  return k ? a[1] : a[0];
}

static __device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
static __device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }

}  // namespace swk
