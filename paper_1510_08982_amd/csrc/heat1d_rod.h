// heat1d_rod.h -- a whole rod resident in registers for all K steps.
//
// Used by the single-rod resident kernel and by the batched persistent kernel.
// The rod occupies local points [0, n) of a block of `nwaves` wavefronts, lane
// l of wavefront w holding points [(64w + l) M, (64w + l + 1) M).  Lane edges
// travel by DPP; wavefront edges are traded through LDS once per step behind a
// barrier, whose kind depends on who holds the rod:
//   kWorkgroup  the whole workgroup (s_barrier);
//   kGroup      a group of wavefronts inside the workgroup, synchronised by an
//               LDS arrival counter (several groups run different rods);
//   kWave       a single wavefront: no barrier at all.
#pragma once

#include "heat1d_device.h"

namespace heat1d {

enum class RodSync { kWorkgroup, kGroup, kWave };

// Barrier of `nwaves` wavefronts sharing the monotone LDS counter *count;
// *epoch counts the barriers this wavefront has passed.
__device__ __forceinline__ void group_barrier(int* count, int nwaves, int* epoch) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(count, 1);
  *epoch += 1;
  const int target = nwaves * *epoch;
  while (uniform(__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) <
         target)
    __builtin_amdgcn_s_sleep(0);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// lds: 4*nwaves elements (two parities x nwaves x {first, last}).
// count/epoch: the group barrier state (kGroup only).
template <typename F, int M, RodSync kSync>
__device__ __forceinline__ void rod_resident(const F* __restrict__ src, F* __restrict__ dst, int n,
                                             int K, F r, F c1, F cN, F* lds, int nwaves, int wave,
                                             int lane, bool aligned, int* count = nullptr,
                                             int* epoch = nullptr) {
  F u[M];
  const int q0 = (wave * kWave + lane) * M;
  load_points<F, M>(u, src, q0, n, aligned);

  // Dirichlet ends (Section 2): point 0 is u[0] of lane 0 of wave 0; point
  // n-1 sits at a wave-uniform (wave, lane, register) position.
  const int qN = n - 1;
  const int wN = qN / (kWave * M);
  const int lN = (qN / M) % kWave;
  const int jN = uniform(qN % M);
  const bool active = wave * kWave * M < n;
  if (wave == 0) u[0] = (lane == 0) ? c1 : u[0];
  if (wave == wN) set_point<F, M>(u, jN, lane == lN, cN);

  for (int k = 0; k < K; ++k) {
    F left, right;
    if constexpr (kSync != RodSync::kWave) {
      F* buf = lds + (k & 1) * 2 * nwaves;
      if (lane == 0) buf[2 * wave] = u[0];
      if (lane == kWave - 1) buf[2 * wave + 1] = u[M - 1];
      if constexpr (kSync == RodSync::kWorkgroup)
        __syncthreads();
      else
        group_barrier(count, nwaves, epoch);
      if (!active) continue;
      left = from_lower_lane(u[M - 1]);
      right = from_upper_lane(u[0]);
      const F lw = wave > 0 ? buf[2 * (wave - 1) + 1] : F(0);
      const F rw = wave + 1 < nwaves ? buf[2 * (wave + 1)] : F(0);
      left = (lane == 0) ? lw : left;
      right = (lane == kWave - 1) ? rw : right;
    } else {
      left = from_lower_lane(u[M - 1]);
      right = from_upper_lane(u[0]);
    }
    lane_step<F, M>(u, left, right, r);
    if (wave == 0) u[0] = (lane == 0) ? c1 : u[0];
    if (wave == wN) set_point<F, M>(u, jN, lane == lN, cN);
  }
  if (active) store_points<F, M>(u, dst, q0, q0, 0, n, aligned);
}

}  // namespace heat1d
