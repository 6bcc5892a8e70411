// Allocation-free force evaluation (sw_forces_noalloc, include/sw.h).
//
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc): the same
// work and the same kernels as sw_forces on a one-box context, with every
// device buffer of that context placed in one file-scope static device array
// instead of hipMalloc'd memory.  Each GPU the library runs on holds its own
// copy of the array until the process ends; its address on a device is taken
// once, with the device current, by hipGetSymbolAddress (the array's name in
// host code is only a host-side stand-in).  Calls on one GPU share the array:
// each call clears what must start at zero with fill kernels, and calls that
// overlap on one GPU race.
#include "sw_ctx.h"

#include <cmath>
#include <mutex>

namespace {

using namespace swk;
using namespace swh;

constexpr size_t kScratchBytes = (size_t)SW_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
constexpr int kNoallocCap = 64;      // row slots per atom (rows never grow here)
constexpr int kNoallocLpa = 16;      // lanes per atom of the moments and force launches

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};   // device address of `scratch` per device

// The scratch array's address on the current device (looked up once per device).
hipError_t scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return e;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

// Bump placement of 256-byte aligned buffers inside [base, base + size).
struct Carver {
  char* base;
  size_t size, used = 0;
  bool full = false;
  hipError_t operator()(void** p, size_t bytes) {
    const size_t at = (used + 255) & ~(size_t)255;
    if (at + bytes > size) {
      full = true;
      *p = nullptr;
      return hipErrorOutOfMemory;
    }
    *p = base + at;
    used = at + bytes;
    return hipSuccess;
  }
};

}  // namespace

extern "C" int sw_forces_noalloc(const float* x, long long n, const double* h_box, const sw_params* params,
                                 float* f, double* energy, double* virial, void* stream) {
  if (!x || !f || !h_box || !params) return SW_EINVAL;
  if (n < 2) return SW_EINVAL;
  if (n > SW_NOALLOC_MAX_ATOMS) return SW_ESCRATCH;
  hipStream_t s = (hipStream_t)stream;
  // the context lives on the host stack; its device buffers are carved from
  // the scratch array
  sw_ctx c;
  const long long off[2] = {0, n};
  const double cutoff = params->a * params->sigma;
  int st = setup_layout(&c, 1, off, h_box, cutoff, SW_NOALLOC_SKIN, kNoallocCap);
  if (st != SW_OK) return st;
  c.tune.lanes_per_atom = kNoallocLpa;
  Phys ph{};
  if ((st = make_phys(&c, params, 1.0, 1.0, &ph)) != SW_OK) return st;
  void* base = nullptr;
  hipError_t e;
  if ((e = scratch_ptr(&base)) != hipSuccess) return SW_EHIP;
  Carver carve{(char*)base, kScratchBytes};
  if ((e = place_buffers(&c, carve)) != hipSuccess || (e = place_capacity_buffers(&c, carve)) != hipSuccess)
    return carve.full ? SW_ESCRATCH : SW_EHIP;
  // layout tables and zeroed state, on the caller's stream
  if ((e = hipMemcpyAsync(c.d_reps, c.reps.data(), sizeof(RepInfo), hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(c.d_tile_rep, c.tile_rep.data(), sizeof(int) * c.tile_rep.size(), hipMemcpyHostToDevice,
                          s)) != hipSuccess ||
      (e = hipMemcpyAsync(c.d_uoff, c.uoff.data(), sizeof(long long) * 2, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(c.d_cell_rank, c.cell_rank.data(), sizeof(int) * c.ctot, hipMemcpyHostToDevice, s)) !=
          hipSuccess)
    return SW_EHIP;
  if ((e = launch_fill_i32(c.d.flags, 0, F_NFLAGS, s)) != hipSuccess ||
      (e = launch_fill_i32(c.d.dflag, 0, 2, s)) != hipSuccess ||
      (e = launch_fill_f64(c.d.thermo_cur, 0.0, kNQ, s)) != hipSuccess)
    return SW_EHIP;
  // sw_forces on a fresh context: sort into internal order, build the rows,
  // moments, forces and sums, scatter back in the caller's order
  if ((e = sort_in(&c, x, nullptr, s)) != hipSuccess) return SW_EHIP;
  if ((e = launch_moments(c.d, ph, kNoallocLpa, 0, 1, 1, s)) != hipSuccess) return SW_EHIP;
  if ((e = launch_forces(c.d, ph, kNoallocLpa, MODE_FORCES, 1, 0, nullptr, s)) != hipSuccess) return SW_EHIP;
  Flags fl;
  if ((e = read_flags(&c, s, &fl)) != hipSuccess) return SW_EHIP;
  if (fl.nbr_over) return SW_ENBR_OVERFLOW;
  if (fl.cell_over) return SW_ECELL_OVERFLOW;
  if ((e = launch_scatter_out(c.d, 0, nullptr, nullptr, (float4*)f, s)) != hipSuccess) return SW_EHIP;
  if ((energy || virial) && (e = launch_copy_thermo(c.d, energy, virial, s)) != hipSuccess) return SW_EHIP;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return SW_EHIP;
  return fl.overlap ? SW_EOVERLAP : SW_OK;
}
