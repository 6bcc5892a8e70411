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

// Hardware id of the XCC (accelerator die, with its own L2) the wavefront
// runs on.
static __device__ __forceinline__ unsigned xcc_id() {
  unsigned v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
  return v & (kMaxXcc - 1);
}

// The compute unit the wavefront runs on, within its XCC: CU_ID, SH_ID
// and SE_ID of the HW_ID register (bits 8..15), one value per CU.
static __device__ __forceinline__ unsigned cu_key() {
  unsigned v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_HW_ID)" : "=s"(v));
  return (v >> 8) & 0xffu;
}

// The thread index through a volatile asm copy: the compiler cannot hoist
// it, or anything computed from it, out of a loop.  A kernel that loops
// over whole steps passes it to each tile it processes, so lane offsets are
// recomputed per tile (a few instructions) instead of being held in
// registers across every phase of the loop.
static __device__ __forceinline__ unsigned opaque_tid() {
  unsigned r;
  asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"((unsigned)__builtin_amdgcn_workitem_id_x()));
  return r;
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

// One DPP exchange of a float: the value of the lane that `ctrl` names.
template <int CTRL>
static __device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

// Sum over each aligned group of W lanes, the same bits in every lane of the
// group (each step adds a pair whose two orders round alike).  Groups of up
// to 16 lanes reduce within their DPP row: neighbours (quad_perm 1,0,3,2),
// pairs (quad_perm 2,3,0,1), quads (row_half_mirror: lane 7 - l of the
// half-row, which holds the other quad's sum), half-rows (row_mirror); wider
// groups add the row-crossing steps by lane shuffles.
template <int W>
static __device__ __forceinline__ float group_sum(float v) {
  if (W >= 2) v += dpp<0xB1>(v);
  if (W >= 4) v += dpp<0x4E>(v);
  if (W >= 8) v += dpp<0x141>(v);
  if (W >= 16) v += dpp<0x140>(v);
#pragma unroll
  for (int m = 16; m < W; m <<= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Inclusive prefix sum over each aligned group of W lanes (lane = index in
// the group).  Groups of up to 16 lanes use DPP row shifts (a source outside
// the group is masked by the lane test); wider groups lane shuffles.
template <int W>
static __device__ __forceinline__ int group_prefix(int v, int lane) {
  if (W > 16) {
#pragma unroll
    for (int o = 1; o < W; o <<= 1) {
      const int u = __shfl_up(v, o, W);
      if (lane >= o) v += u;
    }
    return v;
  }
  if (W > 1) { const int u = __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false); if (lane >= 1) v += u; }
  if (W > 2) { const int u = __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false); if (lane >= 2) v += u; }
  if (W > 4) { const int u = __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false); if (lane >= 4) v += u; }
  if (W > 8) { const int u = __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false); if (lane >= 8) v += u; }
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

// Dual numbers (value, derivative along a tangent direction) and the leg
// geometry of one neighbour in them: the tangent kernels' arithmetic.
struct D {
  float v, d;
};
static __device__ __forceinline__ D operator+(D a, D b) { return {a.v + b.v, a.d + b.d}; }
static __device__ __forceinline__ D operator-(D a, D b) { return {a.v - b.v, a.d - b.d}; }
static __device__ __forceinline__ D operator*(D a, D b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
static __device__ __forceinline__ D operator*(float s, D a) { return {s * a.v, s * a.d}; }
static __device__ __forceinline__ D operator+(D a, float s) { return {a.v + s, a.d}; }
static __device__ __forceinline__ D operator-(D a, float s) { return {a.v - s, a.d}; }
static __device__ __forceinline__ D neg(D a) { return {-a.v, -a.d}; }
static __device__ __forceinline__ D rsqD(D a) {
  const float r = rsq(a.v);
  return {r, -0.5f * r * r * r * a.d};
}
static __device__ __forceinline__ D rcpD(D a) {
  const float r = rcp(a.v);
  return {r, -r * r * a.d};
}
static __device__ __forceinline__ D ex2D(D a) {
  const float e = ex2(a.v);
  return {e, e * 0.69314718055994531f * a.d};
}

struct Leg {
  D ux, uy, uz, r, ir, idr, eg;
};

// Leg geometry of one neighbour as dual numbers: difference dd, tangent dt.
static __device__ __forceinline__ Leg leg_dual(const float3& dd, const float3& dt, const Phys& p) {
  const D dx{dd.x, dt.x}, dy{dd.y, dt.y}, dz{dd.z, dt.z};
  const D r2 = dx * dx + dy * dy + dz * dz;
  Leg G;
  G.ir = rsqD(r2);
  G.r = r2 * G.ir;
  G.ux = dx * G.ir; G.uy = dy * G.ir; G.uz = dz * G.ir;
  G.idr = rcpD(G.r - p.rc);
  G.eg = ex2D(p.gsig_l2e * G.idr);
  return G;
}

static __device__ __forceinline__ float3 sub3(const float4& a, const float4& b) {
  return make_float3(a.x - b.x, a.y - b.y, a.z - b.z);
}

}  // namespace swk
