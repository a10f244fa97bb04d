// Device helpers shared by the kernels: address-space re-typing, the opaque
// thread index and wave-wide reductions on the DPP network.
#pragma once

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

namespace expri {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// Pointers held in the instance descriptors are generic; accesses through
// them compile to flat instructions, which also count against the LDS wait
// counter (an LDS wait then drains in-flight memory loads too).  The hot
// loops re-type them as global-memory pointers first.
#define GMEM __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ GMEM T *gbl(T *p) {
  return (GMEM T *)p;
}

// Read-only data that the kernels never write during a launch (schedules):
// re-typed as constant memory, so that uniform reads become scalar loads,
// counted apart from the vector loads a solve pass keeps in flight.
#define CMEM __attribute__((address_space(4)))

// s_waitcnt operand: vector memory count 0, the other counters unconstrained
constexpr unsigned kWaitVm0 = 0x0F70;
template <class T>
__device__ __forceinline__ const CMEM T *cst(const T *p) {
  return (const CMEM T *)p;
}

// The thread index as an opaque value.  Per-lane values derived from it
// (addresses, masks) are then computed inside each phase instead of being
// hoisted to the kernel entry and held in registers across the whole step.
__device__ __forceinline__ int tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// orders a wave's own LDS traffic (its LDS operations complete in order)
__device__ __forceinline__ void wfence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// Wave-wide reductions on the DPP network: a butterfly inside each 16-lane
// row (pairs of lanes 1 and 2 apart, then the 8- and 16-lane mirrors), then
// the four row results read out in a fixed order.  Every lane ends with the
// bit-identical value.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane i <-> 7 - i in each 8 lanes
constexpr int kDppMirror = 0x140;     // lane i <-> 15 - i in each 16 lanes

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<kDppXor1>(v);
  v += dpp_d<kDppXor2>(v);
  v += dpp_d<kDppHalfMirror>(v);
  v += dpp_d<kDppMirror>(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// max that propagates NaN
__device__ __forceinline__ double nmax(double a, double b) {
  return (isnan(a) || a > b) ? a : b;
}

__device__ __forceinline__ double wave_max(double v) {
  v = nmax(v, dpp_d<kDppXor1>(v));
  v = nmax(v, dpp_d<kDppXor2>(v));
  v = nmax(v, dpp_d<kDppHalfMirror>(v));
  v = nmax(v, dpp_d<kDppMirror>(v));
  return nmax(nmax(readlane_d(v, 0), readlane_d(v, 16)), nmax(readlane_d(v, 32), readlane_d(v, 48)));
}

// sum over aligned groups of G lanes (G a power of two <= 64); the group's
// lanes end with the same value
__device__ __forceinline__ double group_sum(double v, int G) {
  if (G >= 2) v += dpp_d<kDppXor1>(v);
  if (G >= 4) v += dpp_d<kDppXor2>(v);
  if (G >= 8) v += dpp_d<kDppHalfMirror>(v);
  if (G >= 16) v += dpp_d<kDppMirror>(v);
  if (G >= 32) v += __shfl_xor(v, 16, 64);
  if (G >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

}  // namespace expri
