// Wavefront-level reductions through DPP row operations (gfx9 encodings).
#pragma once
#include <hip/hip_runtime.h>

namespace phs {

// Orders the LDS accesses of one wavefront across a point (no workgroup
// barrier): outstanding LDS operations complete, and the compiler moves no
// memory access across it.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// DPP move of a double (both halves), all rows and banks enabled.
template <int CTRL>
__device__ inline double dpp_mov(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, true);
  hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
// Sum over lane groups of G (1, 2, 4, 8 or 16) lanes inside a DPP row; every
// lane of the group receives the group sum.
template <int G>
__device__ inline double group_sum(double v) {
  if (G == 16) {
    v += dpp_mov<0x128>(v);  // row_ror:8: lanes l, l+8 of the row
    v += dpp_mov<0x124>(v);  // row_ror:4: lanes congruent mod 4
  } else if (G == 8) {
    v += dpp_mov<0x141>(v);  // row_half_mirror: lanes l, 7-l of the half row
  }
  if (G >= 4) v += dpp_mov<0x4E>(v);  // quad_perm [2,3,0,1]
  if (G >= 2) v += dpp_mov<0xB1>(v);  // quad_perm [1,0,3,2]
  return v;
}
// Sum over the wave, the same value in every lane: row sums by DPP, then
// the four row sums read from lanes 0, 16, 32, 48 in a fixed order.
__device__ inline double wave_total(double v) {
  v = group_sum<16>(v);
  const int lo = __double2loint(v), hi = __double2hiint(v);
  double r[4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    r[k] = __hiloint2double(__builtin_amdgcn_readlane(hi, 16 * k),
                            __builtin_amdgcn_readlane(lo, 16 * k));
  return (r[0] + r[1]) + (r[2] + r[3]);
}
__device__ inline double wave_max(double v) {
  v = fmax(v, dpp_mov<0x128>(v));
  v = fmax(v, dpp_mov<0x124>(v));
  v = fmax(v, dpp_mov<0x4E>(v));
  v = fmax(v, dpp_mov<0xB1>(v));
  const int lo = __double2loint(v), hi = __double2hiint(v);
  double m = v;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    m = fmax(m, __hiloint2double(__builtin_amdgcn_readlane(hi, 16 * k),
                                 __builtin_amdgcn_readlane(lo, 16 * k)));
  return m;
}

}  // namespace phs
