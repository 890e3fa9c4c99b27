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

// lds: 8*nwaves elements (two parities x nwaves x {first, last} x 2 points).
// count/epoch: the group barrier state (kGroup only).
//
// A rod held by one wavefront takes its neighbours from DPP alone.  A rod held
// by several wavefronts (two or more points per lane) trades the first and last two points of
// every wavefront once per two steps: in the first step each edge lane also
// advances its copy of the neighbour's nearest point (from the copied pair and
// its own edge point, the operands the owner uses, in the same order), so the
// second step finds that neighbour value without an exchange.  One barrier
// per two steps, results bit for bit those of one exchange per step.  The copy
// of the pinned point N-1 (when it is the first point of its wavefront) is
// pinned as well.
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
  // the next wavefront's first point is n-1
  const bool pin_copy = wave + 1 == wN && lN == 0 && jN == 0;
  if (wave == 0) u[0] = (lane == 0) ? c1 : u[0];
  if (wave == wN) set_point<F, M>(u, jN, lane == lN, cN);

  if constexpr (kSync == RodSync::kWave || M < 2) {
    for (int k = 0; k < K; ++k) {
      F left = from_lower_lane(u[M - 1]);
      F right = from_upper_lane(u[0]);
      if constexpr (kSync != RodSync::kWave) {
        // one point per lane: trade the edge points every step
        F* buf = lds + (k & 1) * 2 * nwaves;
        if (lane == 0) buf[2 * wave] = u[0];
        if (lane == kWave - 1) buf[2 * wave + 1] = u[M - 1];
        if constexpr (kSync == RodSync::kWorkgroup)
          __syncthreads();
        else
          group_barrier(count, nwaves, epoch);
        if (!active) continue;
        const F lw = wave > 0 ? buf[2 * (wave - 1) + 1] : F(0);
        const F rw = wave + 1 < nwaves ? buf[2 * (wave + 1)] : F(0);
        left = (lane == 0) ? lw : left;
        right = (lane == kWave - 1) ? rw : right;
      }
      lane_step<F, M>(u, left, right, r);
      if (wave == 0) u[0] = (lane == 0) ? c1 : u[0];
      if (wave == wN) set_point<F, M>(u, jN, lane == lN, cN);
    }
    if (active) store_points<F, M>(u, dst, q0, q0, 0, n, aligned);
    return;
  }
  for (int k = 0; k < K; k += 2) {
    F left, right, left2 = F(0), right2 = F(0);
    {
      F* buf = lds + ((k >> 1) & 1) * 4 * nwaves;
      if (lane == 0) {
        buf[4 * wave] = u[0];
        buf[4 * wave + 1] = u[1];
      }
      if (lane == kWave - 1) {
        buf[4 * wave + 2] = u[M - 1];
        buf[4 * wave + 3] = u[M - 2];
      }
      if constexpr (kSync == RodSync::kWorkgroup)
        __syncthreads();
      else
        group_barrier(count, nwaves, epoch);
      if (!active) continue;
      // the lane shifts first, with every lane active: a DPP shift that the
      // compiler moved under a lane condition would read the excluded lanes
      // as zero (the empty asm keeps it here)
      left = from_lower_lane(u[M - 1]);
      right = from_upper_lane(u[0]);
      asm volatile("" : "+v"(left), "+v"(right));
      // lo1, lo2: points -1, -2 of this wavefront; hi1, hi2: points 64M, 64M+1
      const F lo1 = wave > 0 ? buf[4 * (wave - 1) + 2] : F(0);
      const F lo2 = wave > 0 ? buf[4 * (wave - 1) + 3] : F(0);
      const F hi1 = wave + 1 < nwaves ? buf[4 * (wave + 1)] : F(0);
      const F hi2 = wave + 1 < nwaves ? buf[4 * (wave + 1) + 1] : F(0);
      left = (lane == 0) ? lo1 : left;
      right = (lane == kWave - 1) ? hi1 : right;
      // the copies after one step, as their owners compute them
      left2 = eq3_step(lo2, lo1, u[0], r);
      right2 = pin_copy ? cN : eq3_step(u[M - 1], hi1, hi2, r);
    }
    lane_step<F, M>(u, left, right, r);
    if (wave == 0) u[0] = (lane == 0) ? c1 : u[0];
    if (wave == wN) set_point<F, M>(u, jN, lane == lN, cN);
    if (k + 1 < K) {
      left = from_lower_lane(u[M - 1]);
      right = from_upper_lane(u[0]);
      asm volatile("" : "+v"(left), "+v"(right));
      left = (lane == 0) ? left2 : left;
      right = (lane == kWave - 1) ? right2 : right;
      lane_step<F, M>(u, left, right, r);
      if (wave == 0) u[0] = (lane == 0) ? c1 : u[0];
      if (wave == wN) set_point<F, M>(u, jN, lane == lN, cN);
    }
  }
  if (active) store_points<F, M>(u, dst, q0, q0, 0, n, aligned);
}

}  // namespace heat1d
