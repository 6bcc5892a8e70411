// Forward-mode tangent kernels and the checkpointed discrete adjoint of NVE
// velocity Verlet.
//
// A tangent pass carries (value, derivative) pairs through the same
// moments/forces arithmetic as the force kernels, with every leg vector
// moving as d_ij + eps (w_j - w_i).  One pass along w gives:
//   (dF/dx) w  (= -H w; H is symmetric, so this is also the transposed product),
//   F, the three-body part F3, the virial traces W2, W3 and their derivative
//   along w.
// The parameter derivatives follow from the reduced form of the model
// (Sec. II.A: E depends on sigma and epsilon only through eps E*(x/sigma)):
//   dF/deps = F/eps,  dF/dlambda = F3/lambda,  dF/dsigma = -(1/sigma) dW/dx,
//   dU/deps = U/eps,  dU/dlambda = U3/lambda,  dU/dsigma = W/sigma,
// with W the virial trace.
//
// A loss term aW W(x_s) in the virial trace W needs dW/dx per atom: from the
// reduced form, sigma dF/dsigma = -(F + dF/ds) with dF/ds the tangent of the
// forces under a uniform scaling of every leg, and dW/dx = -sigma dF/dsigma,
// so one scaling pass per frame gives dW/dx = F + dF/ds and dW/ds, whence
// dW/dsigma = -(1/sigma) dW/ds (dW/deps = W/eps, dW/dlambda = W3/lambda).
//
// The adjoint of the velocity-Verlet map (a = 4.184e-4 F / m, J = da/dx):
//   xb = xbar_S; vb = vbar_S; frame(S, dt/2)
//   for s = S-1 .. 0:  vb += dt xb;  frame(s, s > 0 ? dt : dt/2)
//   frame(s, c):  xb += c J(x_s) vb + dl_s/dx_s,  thbar += c vb . da/dtheta + dl_s/dtheta
// One tangent pass along vb at x_s gives every term of a frame.  Positions
// are recomputed per checkpoint segment from a checkpoint of positions,
// full-step velocities and the row state, so the recompute repeats the
// forward kernels exactly.  While a segment is recomputed (or, for the last
// segment, while it first runs) every launch writes the frame's positions and
// cell binning straight into per-frame stores; the reverse sweep runs the
// tangent pass on each stored frame with no copies, carrying its rows from
// frame to frame and rebuilding them from a frame's stored cells when that
// frame's displacement check fails.  The loss terms are summed during the
// reverse sweep.
#include "sw_ctx.h"
#include "sw_device.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace swk {
namespace {

// Kinds of tangent force pass: along w for sw_grad (TK_GRAD), along w with
// the per-atom adjoint update of one frame (TK_ADJ), or along a uniform
// scaling of every leg (TK_SCALE: each leg's tangent is the leg itself), which
// gives the frame's virial gradient dW/dx = F + dF/ds (from the reduced form
// of Sec. II.A, sigma dF/dsigma = -(F + dF/ds)) and dW/ds, so that
// dW/dsigma = -(1/sigma) dW/ds.
enum { TK_GRAD = 0, TK_ADJ = 1, TK_SCALE = 2 };

// Forces and their tangent, virial traces and their tangent; by kind the
// adjoint update of a frame or the virial gradient.
template <int LPA, int KIND>
__global__ __launch_bounds__(kBlock) void k_tan_forces(Dev d, Tan t, Phys p, const float4* __restrict__ w, int par,
                                                       Adj a) {
  constexpr bool ADJ = KIND == TK_ADJ;
  constexpr bool SCALE = KIND == TK_SCALE;
  constexpr int APB = kBlock / LPA;
  static_assert(APB >= kMinAPB, "tangent partials are sized for at least kMinAPB atoms per block");
  __shared__ double red[APB * kTQ];
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int g = threadIdx.x / LPA, lane = threadIdx.x % LPA;
  const int i = bid * APB + g;
  // own records and the first row slot before the replica lookup (padded
  // arrays: padding lanes read in bounds and are masked)
  const uint4 ui = pick(d.u, par)[i];
  const float4 wi = SCALE ? make_float4(0.f, 0.f, 0.f, 0.f) : w[i];
  const float4 gwi = ADJ && a.aW != 0.f ? a.gw[i] : make_float4(0.f, 0.f, 0.f, 0.f);
  const float4* m = d.mom + 3 * (size_t)i;
  const float4* md = t.mdot + 3 * (size_t)i;
  const float4 a0 = m[0], a1 = m[1], a2 = m[2], b0 = md[0], b1 = md[1], b2 = md[2];
  // the next frame's row check (adjoint sweep): its position and the row-build position
  const bool chk = ADJ && a.unext != nullptr;
  const uint4 unx = chk ? a.unext[i] : ui;
  const uint4 urf = chk ? d.uref[i] : ui;
  const int nn_row = d.nn[i];
  const int* row = d.nl + (size_t)i * d.cap;
  int jn = row[min(lane, d.cap - 1)];
  const int rep = d.R == 1 ? 0 : __builtin_amdgcn_readfirstlane(d.tile_rep[i >> 6]);
  const RepInfo& R = d.reps[rep];
  const bool real = i < R.iend;
  const float c0 = p.c0, c02 = p.c0 * p.c0;
  // term weights (sw_grad's term mask; an adjoint frame always takes both):
  // the pair derivative scales the two-body force and virial, the leg factor
  // lambda eps e_j every three-body contribution
  const float m2 = KIND == TK_GRAD ? p.term2 : 1.f, m3 = KIND == TK_GRAD ? p.term3 : 1.f;
  D Tm[6], Vm[3], Sm{0.f, 0.f};
  float E2i = 0.f, E3i = 0.f;
  for (int k = 0; k < 6; ++k) Tm[k] = D{0.f, 0.f};
  for (int k = 0; k < 3; ++k) Vm[k] = D{0.f, 0.f};
  int nn = 0;
  if (real) {
    Tm[0] = {a0.x, b0.x}; Tm[1] = {a0.y, b0.y}; Tm[2] = {a0.z, b0.z}; Tm[3] = {a0.w, b0.w};
    Tm[4] = {a1.x, b1.x}; Tm[5] = {a1.y, b1.y}; Vm[0] = {a1.z, b1.z}; Vm[1] = {a1.w, b1.w};
    Vm[2] = {a2.x, b2.x}; Sm = {a2.y, b2.y};
    E2i = a2.z; E3i = a2.w;
    nn = nn_row;
  }
  D fx{0.f, 0.f}, fy{0.f, 0.f}, fz{0.f, 0.f}, w2{0.f, 0.f}, w3{0.f, 0.f};
  float gx = 0.f, gy = 0.f, gz = 0.f;   // three-body force
  for (int s = lane; s < nn; s += LPA) {
    const int j = jn;
    jn = row[min(s + LPA, nn - 1)];   // the next slot, in flight during this one
    // the neighbour's position, tangent and moments in one batch, read
    // whatever the distance (entries beyond the cutoff are ignored)
    const uint4 uj = pick(d.u, par)[j];
    const float4 wj = SCALE ? make_float4(0.f, 0.f, 0.f, 0.f) : w[j];
    const float4* mj = d.mom + 3 * (size_t)j;
    const float4* mdj = t.mdot + 3 * (size_t)j;
    const float4 na = mj[0], nb = mj[1], nc = mj[2], da = mdj[0], db = mdj[1], dc = mdj[2];
    asm volatile("" ::"v"(uj.x), "v"(wj.x), "v"(na.x), "v"(nb.x), "v"(nc.x), "v"(da.x), "v"(db.x), "v"(dc.x));
    const float3 dd = disp(ui, uj, R.scale[0], R.scale[1], R.scale[2]);
    if (dd.x * dd.x + dd.y * dd.y + dd.z * dd.z < p.rc2) {
      const Leg G = leg_dual(dd, SCALE ? dd : sub3(wj, wi), p);
      const D idr2 = G.idr * G.idr;
      const D e1 = ex2D(p.sig_l2e * G.idr);
      const D sr = p.sig * G.ir, s2 = sr * sr, s4 = s2 * s2;
      const D poly = (p.B * s4) - 1.f;
      const D dphi = m2 * (p.Aeps * (e1 * ((-4.f * p.B) * (s4 * G.ir) - p.sig * (poly * idr2))));
      const D gg = (-p.gsig) * idr2;
      const D Ts0 = Tm[0] + D{na.x, da.x}, Ts1 = Tm[1] + D{na.y, da.y}, Ts2 = Tm[2] + D{na.z, da.z};
      const D Ts3 = Tm[3] + D{na.w, da.w}, Ts4 = Tm[4] + D{nb.x, db.x}, Ts5 = Tm[5] + D{nb.y, db.y};
      const D Dv0 = Vm[0] - D{nb.z, db.z}, Dv1 = Vm[1] - D{nb.w, db.w}, Dv2 = Vm[2] - D{nc.x, dc.x};
      const D Ss = Sm + D{nc.y, dc.y};
      const D y0x = Ts0 * G.ux + Ts3 * G.uy + Ts4 * G.uz;
      const D y0y = Ts3 * G.ux + Ts1 * G.uy + Ts5 * G.uz;
      const D y0z = Ts4 * G.ux + Ts5 * G.uy + Ts2 * G.uz;
      const D uTu = G.ux * y0x + G.uy * y0y + G.uz * y0z;
      const D uDv = G.ux * Dv0 + G.uy * Dv1 + G.uz * Dv2;
      const D q = uTu - (2.f * c0) * uDv + c02 * Ss - (2.f * p.qc) * G.eg;
      const D uy_ = uTu - c0 * uDv;
      const D px = (y0x - c0 * Dv0) - uy_ * G.ux;
      const D py = (y0y - c0 * Dv1) - uy_ * G.uy;
      const D pz = (y0z - c0 * Dv2) - uy_ * G.uz;
      const D le = m3 * (p.lameps * G.eg);
      const D b3 = le * gg * q;
      const D a2 = 2.f * (le * G.ir);
      const D a1 = dphi + b3;
      fx = fx + a1 * G.ux + a2 * px;
      fy = fy + a1 * G.uy + a2 * py;
      fz = fz + a1 * G.uz + a2 * pz;
      gx += b3.v * G.ux.v + a2.v * px.v;
      gy += b3.v * G.uy.v + a2.v * py.v;
      gz += b3.v * G.uz.v + a2.v * pz.v;
      // virial traces: half the pair leg, and the own centre's legs (the
      // tangential part of a leg force has no trace)
      const D ymx = Tm[0] * G.ux + Tm[3] * G.uy + Tm[4] * G.uz - c0 * Vm[0];
      const D ymy = Tm[3] * G.ux + Tm[1] * G.uy + Tm[5] * G.uz - c0 * Vm[1];
      const D ymz = Tm[4] * G.ux + Tm[5] * G.uy + Tm[2] * G.uz - c0 * Vm[2];
      const D uym = G.ux * ymx + G.uy * ymy + G.uz * ymz;
      const D uVm = G.ux * Vm[0] + G.uy * Vm[1] + G.uz * Vm[2];
      const D qown = uym - c0 * uVm + c02 * Sm - p.qc * G.eg;
      w2 = w2 - 0.5f * (G.r * dphi);
      w3 = w3 - le * (G.r * (gg * qown));
    }
  }
  fx.v = group_sum<LPA>(fx.v); fx.d = group_sum<LPA>(fx.d);
  fy.v = group_sum<LPA>(fy.v); fy.d = group_sum<LPA>(fy.d);
  fz.v = group_sum<LPA>(fz.v); fz.d = group_sum<LPA>(fz.d);
  gx = group_sum<LPA>(gx); gy = group_sum<LPA>(gy); gz = group_sum<LPA>(gz);
  w2.v = group_sum<LPA>(w2.v); w2.d = group_sum<LPA>(w2.d);
  w3.v = group_sum<LPA>(w3.v); w3.d = group_sum<LPA>(w3.d);
  if (lane == 0) {
    double q[kTQ] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (real && SCALE) {
      // the virial gradient of this frame, and dW/ds for the sigma derivative
      t.gw[i] = make_float4(fx.v + fx.d, fy.v + fy.d, fz.v + fz.d, 0.f);
      q[7] = (double)w2.d + (double)w3.d;
    } else if (real) {
      d.f[i] = make_float4(fx.v, fy.v, fz.v, 0.f);
      t.fdot[i] = make_float4(fx.d, fy.d, fz.d, 0.f);
      t.f3[i] = make_float4(gx, gy, gz, 0.f);
      q[0] = E2i; q[1] = E3i; q[2] = w2.v; q[3] = w3.v;
      q[4] = (double)wi.x * fx.v + (double)wi.y * fy.v + (double)wi.z * fz.v;
      q[5] = (double)wi.x * gx + (double)wi.y * gy + (double)wi.z * gz;
      q[6] = (double)w2.d + (double)w3.d;
      if (ADJ) {
        const float norm = (float)(1.0 / ((double)R.n * (a.S + 1)));
        float4 xb = a.xb[i];
        xb.x += a.coef_cm * fx.d - (a.aU * fx.v + a.a3 * gx) * norm;
        xb.y += a.coef_cm * fy.d - (a.aU * fy.v + a.a3 * gy) * norm;
        xb.z += a.coef_cm * fz.d - (a.aU * fz.v + a.a3 * gz) * norm;
        if (a.aW != 0.f) {   // + aW dW/dx / (N (S + 1))
          xb.x += a.aW * norm * gwi.x;
          xb.y += a.aW * norm * gwi.y;
          xb.z += a.aW * norm * gwi.z;
        }
        xb.w = 0.f;
        a.xb[i] = xb;
        if (!a.last)
          a.vb_next[i] = make_float4(wi.x + a.dt * xb.x, wi.y + a.dt * xb.y, wi.z + a.dt * xb.z, 0.f);
        if (chk) {
          const float3 dd = disp(urf, unx, R.scale[0], R.scale[1], R.scale[2]);
          if (dd.x * dd.x + dd.y * dd.y + dd.z * dd.z > p.half_skin * p.half_skin)
            d.dflag[(par ^ 1) * d.R + rep] = 1;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kTQ; ++k) red[g * kTQ + k] = q[k];
  }
  __syncthreads();
  if (threadIdx.x < kTQ) {
    double acc = 0.0;
    for (int k = 0; k < APB; ++k) acc += red[k * kTQ + threadIdx.x];
    const size_t slot = (size_t)threadIdx.x * (d.npad / APB) + bid;
    if (ADJ || SCALE) {
      // each block owns its slot: the frames of a sweep add up in frame order
      // (the w.F terms weighted by the frame coefficient; values unweighted)
      a.tacc[slot] += (threadIdx.x >= 4 && threadIdx.x < 7 ? a.coef_d : 1.0) * acc;
    } else {
      t.tpartial[slot] = acc;
    }
  }
}

// What to do with a tangent pass's per-replica sums: sw_grad outputs, or one
// frame's contribution to the parameter adjoint and the loss (frame weight
// coef_cm, loss weights aU, a3 with the 1/(n (S+1)) normalisation).
struct PTerm {
  double lam, eps, sig;
  double m2, m3;          // term weights of the energies in dU (the tangent pass weights the rest)
  double aW;              // loss weight of the virial trace (sums of an adjoint sweep)
  double* wdF;
  double* dU;
  double* thbar;
  double* loss;
  double coef_cm, aU, a3;
  int S;
};

// Per-replica sums of the tangent partials (one block per replica, all
// quantities at once, fixed order), then the parameter terms.
__global__ __launch_bounds__(kBlock) void k_reduce_tan(Dev d, Tan t, int apb, PTerm pt) {
  __shared__ double part[kBlock / 64][kTQ];
  const int nbt = d.npad / apb;
  const int wl = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
  for (int rep = blockIdx.x; rep < d.R; rep += gridDim.x) {
    const RepInfo& R = d.reps[rep];
    double acc[kTQ];
#pragma unroll
    for (int k = 0; k < kTQ; ++k) acc[k] = 0.0;
    for (int b = R.ioff / apb + (int)threadIdx.x; b < R.ipad_end / apb; b += kBlock) {
#pragma unroll
      for (int k = 0; k < kTQ; ++k) acc[k] += t.tpartial[(size_t)k * nbt + b];
    }
#pragma unroll
    for (int k = 0; k < kTQ; ++k)
      for (int m = 32; m >= 1; m >>= 1) acc[k] += __shfl_xor(acc[k], m, 64);
    if (wl == 0) {
#pragma unroll
      for (int k = 0; k < kTQ; ++k) part[wv][k] = acc[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double q[kTQ];
#pragma unroll
      for (int k = 0; k < kTQ; ++k) {
        q[k] = ((part[0][k] + part[1][k]) + part[2][k]) + part[3][k];
        t.tsum[rep * kTQ + k] = q[k];
      }
      const double E2 = q[0], E3 = q[1], W2 = q[2], W3 = q[3], wF = q[4], wF3 = q[5], Wd = q[6], Ws = q[7];
      const double g[3] = {wF3 / pt.lam, wF / pt.eps, -Wd / pt.sig};   // w . dF/d(lambda, eps, sigma)
      const double u[3] = {pt.m3 * E3 / pt.lam, (pt.m2 * E2 + pt.m3 * E3) / pt.eps, (W2 + W3) / pt.sig};
      const double u3[3] = {E3 / pt.lam, E3 / pt.eps, W3 / pt.sig};
      if (pt.wdF) for (int k = 0; k < 3; ++k) pt.wdF[3 * rep + k] = g[k];
      if (pt.dU) for (int k = 0; k < 3; ++k) pt.dU[3 * rep + k] = u[k];
      const double norm = 1.0 / ((double)R.n * (pt.S + 1));
      // the virial trace: dW/dlambda = W3/lambda, dW/deps = W/eps, dW/dsigma = -(1/sigma) dW/ds
      const double uw[3] = {W3 / pt.lam, (W2 + W3) / pt.eps, -Ws / pt.sig};
      if (pt.thbar)
        for (int k = 0; k < 3; ++k)
          pt.thbar[3 * rep + k] += pt.coef_cm * g[k] + norm * (pt.aU * u[k] + pt.a3 * u3[k] + pt.aW * uw[k]);
      if (pt.loss) pt.loss[rep] += norm * (pt.aU * (E2 + E3) + pt.a3 * E3 + pt.aW * (W2 + W3));
    }
    __syncthreads();
  }
}

__global__ void k_gather_vec(Dev d, const float4* __restrict__ user, float4* __restrict__ internal) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= d.npad) return;
  const int k = d.ids[i];
  float4 a = k >= 0 && user ? user[k] : make_float4(0.f, 0.f, 0.f, 0.f);
  a.w = 0.f;
  internal[i] = a;
}

__global__ void k_scatter_vec(Dev d, const float4* __restrict__ internal, float4* __restrict__ user) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= d.npad) return;
  const int k = d.ids[i];
  if (k < 0) return;
  float4 a = internal[i];
  a.w = 0.f;
  user[k] = a;
}

template <class T>
__global__ void k_copy(const T* __restrict__ src, T* __restrict__ dst, int n) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

inline unsigned nb(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <int LPA>
hipError_t tan_launch(const Dev& d, const Tan& t, const Phys& p, const float4* w, int par, const Adj* adj,
                      const PTerm& pt, hipStream_t s, bool scale) {
  constexpr int APB = kBlock / LPA;
  const unsigned grid = (unsigned)(d.npad / APB);
  Adj a = adj ? *adj : Adj{};
  if (scale) {   // the frame's virial gradient; its dW/ds joins the sweep's sums
    hipLaunchKernelGGL((k_tan_forces<LPA, TK_SCALE>), dim3(grid), dim3(kBlock), 0, s, d, t, p, w, par, a);
  } else if (adj) {   // an adjoint frame accumulates; the sweep reduces once at its end
    hipLaunchKernelGGL((k_tan_forces<LPA, TK_ADJ>), dim3(grid), dim3(kBlock), 0, s, d, t, p, w, par, a);
  } else {
    hipLaunchKernelGGL((k_tan_forces<LPA, TK_GRAD>), dim3(grid), dim3(kBlock), 0, s, d, t, p, w, par, a);
    hipLaunchKernelGGL(k_reduce_tan, dim3((unsigned)std::min(d.R, 4096)), dim3(kBlock), 0, s, d, t, APB, pt);
  }
  return hipGetLastError();
}

// Per-replica sums of t.tpartial (block partials of a force launch at lpa
// lanes per atom, or a sweep's accumulated sums) and the parameter terms of pt.
hipError_t launch_tan_reduce(const Dev& d, const Tan& t, int lpa, const PTerm& pt, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_tan, dim3((unsigned)std::min(d.R, 4096)), dim3(kBlock), 0, s, d, t, kBlock / lpa, pt);
  return hipGetLastError();
}

// Tangent forces, then (outside an adjoint sweep) the per-replica sums and
// the parameter terms of pt; with scale, the scaling pass of an adjoint frame.
hipError_t launch_tan_forces(const Dev& d, const Tan& t, const Phys& p, int lpa, const float4* w, int par,
                             const Adj* adj, const PTerm& pt, hipStream_t s, bool scale = false) {
  switch (lpa) {
    case 4: return tan_launch<4>(d, t, p, w, par, adj, pt, s, scale);
    case 8: return tan_launch<8>(d, t, p, w, par, adj, pt, s, scale);
    case 16: return tan_launch<16>(d, t, p, w, par, adj, pt, s, scale);
    case 32: return tan_launch<32>(d, t, p, w, par, adj, pt, s, scale);
    case 64: return tan_launch<64>(d, t, p, w, par, adj, pt, s, scale);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_gather_vec(const Dev& d, const float4* user, float4* internal, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_vec, dim3(nb(d.npad)), dim3(kBlock), 0, s, d, user, internal);
  return hipGetLastError();
}

hipError_t launch_scatter_vec(const Dev& d, const float4* internal, float4* user, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter_vec, dim3(nb(d.npad)), dim3(kBlock), 0, s, d, internal, user);
  return hipGetLastError();
}

hipError_t launch_copy_u(const Dev& d, const uint4* src, uint4* dst, hipStream_t s) {
  hipLaunchKernelGGL((k_copy<uint4>), dim3(nb(d.npad)), dim3(kBlock), 0, s, src, dst, d.npad);
  return hipGetLastError();
}

hipError_t launch_copy_v(const Dev& d, const float4* src, float4* dst, hipStream_t s) {
  hipLaunchKernelGGL((k_copy<float4>), dim3(nb(d.npad)), dim3(kBlock), 0, s, src, dst, d.npad);
  return hipGetLastError();
}

}  // namespace swk

using namespace swk;
using namespace swh;

namespace {

// Device buffers of one sw_adjoint call.
// The adjoint's work buffers, held by the context between calls: the k-th
// request of a call gets slot k, reallocated only when it must grow (no
// allocation or free, and so no device synchronisation, once sizes settle).
struct AdjBuffers {
  sw_ctx* c;
  size_t k = 0;
  template <class T>
  hipError_t get(T** p, size_t n) {
    const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    if (k == c->adj_buf.size()) {
      c->adj_buf.push_back(nullptr);
      c->adj_bytes.push_back(0);
    }
    if (c->adj_bytes[k] < bytes) {
      if (c->adj_buf[k]) (void)hipFree(c->adj_buf[k]);
      c->adj_buf[k] = nullptr;
      c->adj_bytes[k] = 0;
      hipError_t e = hipMalloc(&c->adj_buf[k], bytes);
      if (e != hipSuccess) return e;
      c->adj_bytes[k] = bytes;
    }
    *p = (T*)c->adj_buf[k++];
    return hipSuccess;
  }
};

// Per-frame stores of one segment (frames 0..K): positions and the cell
// binning of each frame's positions.
struct FrameStore {
  uint4* u;      // [K+1][Npad]
  int* cnt;      // [K+1][cells]
  uint4* cells;  // [K+1][cells][cell capacity]
};

// The context's device view for frame k of a stored segment of len steps:
// the frame's positions and cells in the parity slot the step reads, the
// next frame's in the slot it writes (the moments launch clears those
// counts, the force launch bins into them).  Without a store: the context's
// own ping-pong arrays.
Dev frame_dev(const sw_ctx* c, const FrameStore* fs, int k, int len) {
  Dev d = c->d;
  if (!fs) return d;
  const int par = k & 1;
  const size_t np = c->npad, nc = c->ctot, ncm = (size_t)c->ctot * c->cc;
  d.u[par] = fs->u + (size_t)k * np;
  d.gcnt[par] = fs->cnt + (size_t)k * nc;
  d.gmem[par] = fs->cells + (size_t)k * ncm;
  if (k < len) {
    d.u[par ^ 1] = fs->u + (size_t)(k + 1) * np;
    d.gcnt[par ^ 1] = fs->cnt + (size_t)(k + 1) * nc;
    d.gmem[par ^ 1] = fs->cells + (size_t)(k + 1) * ncm;
  }
  return d;
}

// len steps of NVE velocity Verlet from positions x_c, full-step velocities
// and the rows in force at x_c.  The first segment of a trajectory builds its
// rows; later segments continue with the rows they inherit, so the step
// sequence, and every rebuild decision, is the same for any checkpoint
// interval.  Ends on the full-step velocity.  Without a store the positions
// start and end in u[0]; with one they start in frame 0 of the store and
// every frame's positions and cells stay there.
hipError_t run_segment(sw_ctx* c, const Phys& ph, int lpa, int len, bool first, const FrameStore* fs,
                       hipStream_t s) {
  hipError_t e;
  const Dev d0 = frame_dev(c, fs, 0, len);
  if ((e = launch_fill_i32(d0.gcnt[0], 0, c->ctot, s)) != hipSuccess) return e;
  if ((e = launch_fill_i32(d0.dflag, 0, 2 * c->R, s)) != hipSuccess) return e;
  if ((e = launch_bin(d0, 0, 0, 0.f, 0.f, s)) != hipSuccess) return e;
  if ((e = launch_moments(d0, ph, lpa, 0, first ? 1 : 0, 0, s)) != hipSuccess) return e;
  if (len == 0) return launch_forces(d0, ph, lpa, MODE_FORCES, 0, 0, nullptr, s);
  if ((e = launch_forces(d0, ph, lpa, MODE_START, 0, 0, nullptr, s)) != hipSuccess) return e;
  for (int t = 1; t <= len; ++t) {
    const int par = t & 1;
    const Dev dt = frame_dev(c, fs, t, len);
    if ((e = launch_moments(dt, ph, lpa, par, 0, 0, s)) != hipSuccess) return e;
    const int mode = t == len ? MODE_NVE_LAST : MODE_NVE;
    if ((e = launch_forces(dt, ph, lpa, mode, 0, par, nullptr, s)) != hipSuccess) return e;
  }
  if (!fs && (len & 1)) return launch_copy_u(c->d, c->d.u[1], c->d.u[0], s);
  return hipSuccess;
}

// Checkpoint of the integrator state at a segment start: positions,
// velocities and the row state (rows, lengths, build positions).
struct Ckpt {
  uint4* u;
  float4* v;
  int* nl;
  int* nn;
  uint4* uref;
};

hipError_t save_ckpt(sw_ctx* c, const Ckpt& k, hipStream_t s) {
  const size_t np = c->npad;
  hipError_t e;
  if ((e = launch_copy_u(c->d, c->d.u[0], k.u, s)) != hipSuccess) return e;
  if ((e = launch_copy_v(c->d, c->d.v, k.v, s)) != hipSuccess) return e;
  if ((e = launch_copy_u(c->d, c->d.uref, k.uref, s)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(k.nn, c->d.nn, sizeof(int) * np, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
  return hipMemcpyAsync(k.nl, c->d.nl, sizeof(int) * np * c->cap, hipMemcpyDeviceToDevice, s);
}

// Restores a checkpoint; its positions go to u_dst.  The first segment's
// checkpoint holds no row state (that segment builds its rows).
hipError_t load_ckpt(sw_ctx* c, const Ckpt& k, uint4* u_dst, bool rows, hipStream_t s) {
  const size_t np = c->npad;
  hipError_t e;
  if ((e = launch_copy_u(c->d, k.u, u_dst, s)) != hipSuccess) return e;
  if ((e = launch_copy_v(c->d, k.v, c->d.v, s)) != hipSuccess) return e;
  if (!rows) return hipSuccess;
  if ((e = launch_copy_u(c->d, k.uref, c->d.uref, s)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(c->d.nn, k.nn, sizeof(int) * np, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
  return hipMemcpyAsync(c->d.nl, k.nl, sizeof(int) * np * c->cap, hipMemcpyDeviceToDevice, s);
}

// Row state only (rows, lengths, build positions) to and from k.
hipError_t save_rows(sw_ctx* c, const Ckpt& k, hipStream_t s) {
  const size_t np = c->npad;
  hipError_t e;
  if ((e = launch_copy_u(c->d, c->d.uref, k.uref, s)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(k.nn, c->d.nn, sizeof(int) * np, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
  return hipMemcpyAsync(k.nl, c->d.nl, sizeof(int) * np * c->cap, hipMemcpyDeviceToDevice, s);
}

hipError_t load_rows(sw_ctx* c, const Ckpt& k, hipStream_t s) {
  const size_t np = c->npad;
  hipError_t e;
  if ((e = launch_copy_u(c->d, k.uref, c->d.uref, s)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(c->d.nn, k.nn, sizeof(int) * np, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
  return hipMemcpyAsync(c->d.nl, k.nl, sizeof(int) * np * c->cap, hipMemcpyDeviceToDevice, s);
}

// Tangent pass along w at the positions of dv.u[par], whose cells are binned
// in dv.gcnt[par] / dv.gmem[par]: moments with energies and their tangent
// (rows rebuilt there when forced or flagged in dv.dflag[par]), then tangent
// forces with the adjoint update of *adj and the per-replica terms of pt.
hipError_t tangent_frame(sw_ctx* c, const Dev& dv, const Phys& ph, int lpa, int par, int force_rebuild,
                         const float4* w, const Adj* adj, const PTerm& pt, hipStream_t s) {
  hipError_t e;
  if ((e = launch_moments_tan(dv, ph, lpa, par, force_rebuild, w, c->t.mdot, s)) != hipSuccess) return e;
  return launch_tan_forces(dv, c->t, ph, lpa, w, par, adj, pt, s);
}

// Scaling pass of an adjoint frame with a virial term in the loss: moments
// and forces with their tangent along a uniform scaling of every leg, which
// leave the frame's virial gradient in c->t.gw and add dW/ds to the sweep's
// sums.  The rows are rebuilt here when the frame's flag asks for it, and
// the flag is then cleared, so the frame's tangent pass that follows reads
// the same rows without building them again.
hipError_t scale_frame(sw_ctx* c, const Dev& dv, const Phys& ph, int lpa, int par, const Adj* adj, hipStream_t s) {
  hipError_t e;
  if ((e = launch_moments_tan(dv, ph, lpa, par, 0, nullptr, c->t.mdot, s)) != hipSuccess) return e;
  if ((e = launch_tan_forces(dv, c->t, ph, lpa, nullptr, par, adj, PTerm{}, s, true)) != hipSuccess) return e;
  return launch_fill_i32(dv.dflag + (size_t)par * dv.R, 0, dv.R, s);
}

// Tangent pass at positions u[0] along w; rows rebuilt first, or kept when
// no atom has moved half the skin since they were built (the skin scaled by
// any change of the box since the build).
hipError_t tangent_pass(sw_ctx* c, const Phys& ph, int lpa, const float4* w, const PTerm& pt, hipStream_t s,
                        bool rebuild) {
  const Dev& d = c->d;
  hipError_t e;
  if ((e = launch_fill_i32(d.gcnt[0], 0, c->ctot, s)) != hipSuccess) return e;
  if ((e = launch_fill_i32(d.dflag, 0, 2 * c->R, s)) != hipSuccess) return e;
  if ((e = launch_bin(d, 0, rebuild ? 0 : 1, (float)(c->cutoff + c->skin), ph.rc, s)) != hipSuccess) return e;
  if ((e = launch_moments_tan(d, ph, lpa, 0, rebuild ? 1 : 0, w, c->t.mdot, s)) != hipSuccess) return e;
  return launch_tan_forces(d, c->t, ph, lpa, w, 0, nullptr, pt, s);
}

}  // namespace

extern "C" {

int sw_grad(sw_ctx* ctx, const float* x, const float* w, const sw_params* params, int term_mask, float* hvp,
            double* wdF, double* dU, void* stream) {
  if (!ctx || !x || !w || !hvp) return SW_EINVAL;
  if (term_mask < 1 || term_mask > (SW_TERM_TWO_BODY | SW_TERM_THREE_BODY)) return SW_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  Phys ph{};
  int st = make_phys(ctx, params, 1.0, 1.0, &ph);
  if (st != SW_OK) return st;
  ph.term2 = (term_mask & SW_TERM_TWO_BODY) ? 1.f : 0.f;
  ph.term3 = (term_mask & SW_TERM_THREE_BODY) ? 1.f : 0.f;
  const int lpa = lpa_for(ctx);
  const PTerm pt{params->lambda, params->epsilon, params->sigma, (double)ph.term2, (double)ph.term3, 0.0,
                 wdF, dU, nullptr, nullptr, 0.0, 0.0, 0.0, 0};
  for (int attempt = 0; attempt < 6; ++attempt) {
    hipError_t e;
    if ((e = reset_flags(ctx, s)) != hipSuccess) return fail_hip(ctx, e);
    bool rebuild = false;
    if (!ctx->have_order) {
      if ((e = sort_in(ctx, x, nullptr, s)) != hipSuccess) return fail_hip(ctx, e);
      rebuild = true;
    } else if ((e = launch_gather_ids(ctx->d, (const float4*)x, 0, s)) != hipSuccess) {
      return fail_hip(ctx, e);
    }
    if ((e = launch_gather_vec(ctx->d, (const float4*)w, ctx->t.w, s)) != hipSuccess) return fail_hip(ctx, e);
    if ((e = tangent_pass(ctx, ph, lpa, ctx->t.w, pt, s, rebuild)) != hipSuccess) return fail_hip(ctx, e);
    Flags fl;
    if ((e = read_flags(ctx, s, &fl)) != hipSuccess) return fail_hip(ctx, e);
    if (fl.nbr_over || fl.cell_over) {
      if ((st = grow(ctx, fl)) != SW_OK) return st;
      continue;
    }
    if ((e = launch_scatter_vec(ctx->d, ctx->t.fdot, (float4*)hvp, s)) != hipSuccess) return fail_hip(ctx, e);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail_hip(ctx, e);
    return fl.overlap ? SW_EOVERLAP : SW_OK;
  }
  return SW_ENBR_OVERFLOW;
}

int sw_adjoint(sw_ctx* ctx, const float* x0, const float* v0, const sw_params* params, double mass, double dt,
               int nsteps, int ckpt_every, double aU, double a3, double aW, const float* xbar_S,
               const float* vbar_S, double* loss, float* xbar0, float* vbar0, double* thbar, float* xS, float* vS,
               void* stream) {
  if (!ctx || !x0 || !v0 || !loss || !xbar0 || !vbar0 || !thbar) return SW_EINVAL;
  if (!(mass > 0.0) || !(dt > 0.0) || nsteps < 0 || ckpt_every <= 0 || !std::isfinite(aU) || !std::isfinite(a3) ||
      !std::isfinite(aW))
    return SW_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  Phys ph{};
  int st = make_phys(ctx, params, mass, dt, &ph);
  if (st != SW_OK) return st;
  const int lpa = lpa_for(ctx);
  const int S = nsteps, K = std::min(ckpt_every, std::max(S, 1));
  const int nseg = S == 0 ? 1 : (S + K - 1) / K;
  const size_t np = ctx->npad;
  const double c_m = kAcc / mass;
  for (int attempt = 0; attempt < 6; ++attempt) {
    AdjBuffers B{ctx};
    uint4 *ck_u = nullptr, *ck_uref = nullptr, *fs_u = nullptr, *fs_cells = nullptr, *st_u = nullptr;
    uint4* rs_uref = nullptr;
    float4 *ck_v = nullptr, *xb = nullptr, *vb[2] = {nullptr, nullptr}, *st_v = nullptr;
    int *ck_nl = nullptr, *ck_nn = nullptr, *fs_cnt = nullptr, *rs_nl = nullptr, *rs_nn = nullptr, *rfl = nullptr;
    double *thb = nullptr, *tacc = nullptr, *lossb = nullptr;
    hipError_t e;
    const size_t nf = (size_t)K + 1;
    if ((e = B.get(&ck_u, np * nseg)) != hipSuccess || (e = B.get(&ck_v, np * nseg)) != hipSuccess ||
        (e = B.get(&ck_uref, np * nseg)) != hipSuccess || (e = B.get(&ck_nn, np * nseg)) != hipSuccess ||
        (e = B.get(&ck_nl, np * ctx->cap * nseg)) != hipSuccess || (e = B.get(&fs_u, np * nf)) != hipSuccess ||
        (e = B.get(&fs_cnt, (size_t)ctx->ctot * nf)) != hipSuccess ||
        (e = B.get(&fs_cells, (size_t)ctx->ctot * ctx->cc * nf)) != hipSuccess ||
        (e = B.get(&xb, np)) != hipSuccess || (e = B.get(&vb[0], np)) != hipSuccess ||
        (e = B.get(&vb[1], np)) != hipSuccess || (e = B.get(&thb, (size_t)ctx->R * 3)) != hipSuccess ||
        (e = B.get(&tacc, (np / kMinAPB + 1) * kTQ)) != hipSuccess || (e = B.get(&lossb, (size_t)ctx->R)) != hipSuccess ||
        (e = B.get(&st_u, np)) != hipSuccess || (e = B.get(&st_v, np)) != hipSuccess ||
        (e = B.get(&rs_nl, np * ctx->cap)) != hipSuccess || (e = B.get(&rs_nn, np)) != hipSuccess ||
        (e = B.get(&rs_uref, np)) != hipSuccess || (e = B.get(&rfl, 2 * (size_t)ctx->R)) != hipSuccess)
      return e == hipErrorOutOfMemory ? SW_ENOMEM : fail_hip(ctx, e);
    const FrameStore fs{fs_u, fs_cnt, fs_cells};
    // caller inputs into internal order (eager: the core below touches only
    // buffers the context owns, so a captured core serves any caller tensors)
    if ((e = reset_flags(ctx, s)) != hipSuccess) return fail_hip(ctx, e);
    if ((e = sort_in(ctx, x0, v0, s)) != hipSuccess) return fail_hip(ctx, e);
    if ((e = launch_gather_vec(ctx->d, (const float4*)xbar_S, xb, s)) != hipSuccess) return fail_hip(ctx, e);
    if ((e = launch_gather_vec(ctx->d, (const float4*)vbar_S, vb[0], s)) != hipSuccess) return fail_hip(ctx, e);
    auto ckpt = [&](int j) {
      return Ckpt{ck_u + (size_t)j * np, ck_v + (size_t)j * np, ck_nl + (size_t)j * np * ctx->cap,
                  ck_nn + (size_t)j * np, ck_uref + (size_t)j * np};
    };
    // The core: forward, final state staged, reverse sweep, sums of all frames.
    auto core = [&](hipStream_t q) -> hipError_t {
      hipError_t r;
      // forward with a checkpoint at every segment start; the last segment
      // runs into the frame store, so the reverse sweep needs no recompute of it
      for (int j = 0; j < nseg; ++j) {
        const int c = j * K, len = std::min(K, S - c);
        if (j > 0 && (r = save_ckpt(ctx, ckpt(j), q)) != hipSuccess) return r;
        if (j == 0) {   // rows of the first segment are built by run_segment itself
          if ((r = launch_copy_u(ctx->d, ctx->d.u[0], ck_u, q)) != hipSuccess) return r;
          if ((r = launch_copy_v(ctx->d, ctx->d.v, ck_v, q)) != hipSuccess) return r;
        }
        const bool last = j == nseg - 1;
        if (last && (r = launch_copy_u(ctx->d, ctx->d.u[0], fs.u, q)) != hipSuccess) return r;
        if ((r = run_segment(ctx, ph, lpa, len, j == 0, last ? &fs : nullptr, q)) != hipSuccess) return r;
      }
      // Row or cell overflow in the forward run is read with the flags at the
      // end (truncated rows and cells stay in bounds); the call then reruns
      // with grown capacities, so the host never waits in between.
      const int len_last = S - (nseg - 1) * K;
      if ((r = launch_copy_u(ctx->d, fs.u + (size_t)len_last * np, st_u, q)) != hipSuccess) return r;
      if ((r = launch_copy_v(ctx->d, ctx->d.v, st_v, q)) != hipSuccess) return r;
      // Reverse sweep.  Its rows start as the forward run's final rows (valid
      // at x_S) and go from frame to frame like the forward's: a frame
      // rebuilds them (from its stored cells) only when some atom of it lies
      // more than half the skin from the rows' build position, which the
      // previous frame's tangent-force launch checks.  They are set aside
      // while a segment is recomputed, so the rebuilds, and every sum, depend
      // on the frames alone and not on where segments start.
      int cur = 0;
      if ((r = launch_fill_f64(thb, 0.0, 3 * (long long)ctx->R, q)) != hipSuccess) return r;
      if ((r = launch_fill_f64(lossb, 0.0, ctx->R, q)) != hipSuccess) return r;
      if ((r = launch_fill_f64(tacc, 0.0, (long long)(np / kMinAPB + 1) * kTQ, q)) != hipSuccess) return r;
      if ((r = launch_fill_i32(rfl, 0, 2 * ctx->R, q)) != hipSuccess) return r;
      for (int j = nseg - 1; j >= 0; --j) {
        const int c = j * K, len = std::min(K, S - c);
        if (j < nseg - 1) {   // recompute the segment into the frame store
          const Ckpt rows{nullptr, nullptr, rs_nl, rs_nn, rs_uref};
          if ((r = save_rows(ctx, rows, q)) != hipSuccess) return r;
          if ((r = load_ckpt(ctx, ckpt(j), fs.u, j > 0, q)) != hipSuccess) return r;
          if ((r = run_segment(ctx, ph, lpa, len, j == 0, &fs, q)) != hipSuccess) return r;
          if ((r = load_rows(ctx, rows, q)) != hipSuccess) return r;
        }
        const int s_lo = j == 0 ? 0 : c + 1;
        for (int sf = c + len; sf >= s_lo; --sf) {
          const int k = sf - c, par = sf & 1;
          Dev dv = ctx->d;   // frame sf: its positions and cells in parity slot sf & 1
          dv.u[par] = fs.u + (size_t)k * np;
          dv.gcnt[par] = fs.cnt + (size_t)k * ctx->ctot;
          dv.gmem[par] = fs.cells + (size_t)k * ctx->ctot * ctx->cc;
          dv.dflag = rfl;
          dv.sync_rb = 0;   // the sweep's own per-replica flags
          const double coef = (sf == S || sf == 0) ? 0.5 * dt : dt;
          // frame sf - 1 is frame k - 1 of this store (a store holds its segment's start)
          const Adj a{xb, vb[cur ^ 1], (float)(coef * c_m), (float)dt, (float)aU, (float)a3, S, sf == 0,
                      coef * c_m, tacc, sf > 0 ? fs.u + (size_t)(k - 1) * np : nullptr, (float)aW, ctx->t.gw};
          if (aW != 0.0 && (r = scale_frame(ctx, dv, ph, lpa, par, &a, q)) != hipSuccess) return r;
          if ((r = tangent_frame(ctx, dv, ph, lpa, par, 0, vb[cur], &a, PTerm{}, q)) != hipSuccess) return r;
          if (sf > 0) cur ^= 1;
        }
      }
      // parameter adjoint and loss from the sums of all frames (weights already applied)
      Tan tr = ctx->t;
      tr.tpartial = tacc;
      const PTerm pt{params->lambda, params->epsilon, params->sigma, 1.0, 1.0, aW, nullptr, nullptr, thb, lossb, 1.0,
                     aU, a3, S};
      return launch_tan_reduce(ctx->d, tr, lpa, pt, q);
    };
    if (ctx->tune.graph_steps > 0) {
      // replay a captured core when everything it reads is unchanged
      const double sc[10] = {aU, a3, aW, dt, mass, c_m, params->lambda, params->epsilon, params->sigma, (double)S};
      const int meta[5] = {K, nseg, lpa, ctx->alloc_gen, ctx->R};
      std::vector<unsigned char> key(sizeof(Dev) + sizeof(Tan) + sizeof(Phys) + sizeof sc + sizeof meta +
                                     sizeof(void*) * ctx->adj_buf.size());
      unsigned char* kp = key.data();
      std::memcpy(kp, &ctx->d, sizeof(Dev)); kp += sizeof(Dev);
      std::memcpy(kp, &ctx->t, sizeof(Tan)); kp += sizeof(Tan);
      std::memcpy(kp, &ph, sizeof(Phys)); kp += sizeof(Phys);
      std::memcpy(kp, sc, sizeof sc); kp += sizeof sc;
      std::memcpy(kp, meta, sizeof meta); kp += sizeof meta;
      std::memcpy(kp, ctx->adj_buf.data(), sizeof(void*) * ctx->adj_buf.size());
      if (!(ctx->adj_gexec && key == ctx->adj_gkey)) {
        if (ctx->adj_gexec) { (void)hipGraphExecDestroy(ctx->adj_gexec); ctx->adj_gexec = nullptr; }
        if (ctx->adj_graph) { (void)hipGraphDestroy(ctx->adj_graph); ctx->adj_graph = nullptr; }
        ctx->adj_gkey.clear();
        if (!ctx->cap_stream && (e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking)) != hipSuccess)
          return fail_hip(ctx, e);
        if ((e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
          return fail_hip(ctx, e);
        const hipError_t ce = core(ctx->cap_stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(ctx->cap_stream, &g);
        if (ce != hipSuccess || e != hipSuccess) {
          if (g) (void)hipGraphDestroy(g);
          return fail_hip(ctx, ce != hipSuccess ? ce : e);
        }
        if ((e = hipGraphInstantiate(&ctx->adj_gexec, g, nullptr, nullptr, 0)) != hipSuccess) {
          (void)hipGraphDestroy(g);
          ctx->adj_gexec = nullptr;
          return fail_hip(ctx, e);
        }
        ctx->adj_graph = g;
        ctx->adj_gkey = key;
      }
      if ((e = hipGraphLaunch(ctx->adj_gexec, s)) != hipSuccess) return fail_hip(ctx, e);
    } else if ((e = core(s)) != hipSuccess) {
      return fail_hip(ctx, e);
    }
    // results back to caller order
    {
      Dev dS = ctx->d;
      dS.u[0] = st_u;
      dS.v = st_v;
      if ((xS || vS) && (e = launch_scatter_out(dS, 0, (float4*)xS, (float4*)vS, nullptr, s)) != hipSuccess)
        return fail_hip(ctx, e);
    }
    const int cur = S & 1;   // one swap per frame s > 0
    if ((e = launch_scatter_vec(ctx->d, xb, (float4*)xbar0, s)) != hipSuccess) return fail_hip(ctx, e);
    if ((e = launch_scatter_vec(ctx->d, vb[cur], (float4*)vbar0, s)) != hipSuccess) return fail_hip(ctx, e);
    if ((e = hipMemcpyAsync(thbar, thb, sizeof(double) * 3 * ctx->R, hipMemcpyDeviceToDevice, s)) != hipSuccess)
      return fail_hip(ctx, e);
    if ((e = hipMemcpyAsync(loss, lossb, sizeof(double) * ctx->R, hipMemcpyDeviceToDevice, s)) != hipSuccess)
      return fail_hip(ctx, e);
    Flags fl;
    if ((e = read_flags(ctx, s, &fl)) != hipSuccess) return fail_hip(ctx, e);
    if (fl.nbr_over || fl.cell_over) {
      if ((st = grow(ctx, fl)) != SW_OK) return st;
      continue;
    }
    ctx->steps += 2 * (long long)S;
    return fl.overlap ? SW_EOVERLAP : SW_OK;
  }
  return SW_ENBR_OVERFLOW;
}

}  // extern "C"
