// heat1d_rod.h -- a whole rod resident in registers for all K steps.
//
// Used by the single-rod resident kernel and by the batched persistent kernel.
// The rod occupies local points [0, n) of a block of `nwaves` wavefronts
// (kWG = true: a workgroup, neighbouring wavefronts exchange their edge points
// through LDS once per step behind one barrier) or of a single wavefront
// (kWG = false: no barrier at all, lane edges travel by DPP only).
#pragma once

#include "heat1d_device.h"

namespace heat1d {

// lds: 4*nwaves elements (two parities x nwaves x {first, last}).
template <typename F, int M, bool kWG>
__device__ __forceinline__ void rod_resident(const F* __restrict__ src, F* __restrict__ dst, int n,
                                             int K, F r, F c1, F cN, F* lds, int nwaves, int wave,
                                             int lane, bool aligned) {
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
    if constexpr (kWG) {
      F* buf = lds + (k & 1) * 2 * nwaves;
      if (lane == 0) buf[2 * wave] = u[0];
      if (lane == kWave - 1) buf[2 * wave + 1] = u[M - 1];
      __syncthreads();
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
