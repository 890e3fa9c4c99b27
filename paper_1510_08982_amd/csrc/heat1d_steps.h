// heat1d_steps.h -- register sweeps shared by the tiled, pipelined and wide
// synchronous kernels: fused S-step sweeps and the host-side weights of the
// S-step stencil.
#pragma once

#include "heat1d_device.h"
#include "heat1d_weights.h"

namespace heat1d {

// Fused steps.  S steps of Eq.3 on points away from the rod ends equal one
// application of the S-step stencil u_i <- w_0 u_i + sum_{d=1..S} w_d
// (u_{i-d} + u_{i+d}), whose weights are the coefficients of the S-th power of
// the three-point stencil (r, 1-2r, r) (all positive for r <= 1/2).  Per point
// that is S additions, one multiplication and S fused multiply-adds, 2 + 1/S
// instructions per point update instead of 3, with fewer roundings.  The
// garbage entering a tile at its two cut edges still advances one point per
// step, so the halo rule H >= steps is unchanged.  The weights come from
// step_weights() in heat1d_weights.h.

// S fused steps of the lane's M points from u into v (a second register set).
// Out of place, the compiler can order the work freely without copying
// registers back at the end of a sweep; the caller alternates u -> v -> u.
// The lower lane's last S points and the upper lane's first S points come by
// DPP.  Smallest weights first.
// The sweep itself, given the S points left of the lane (lo[d] = point -1-d)
// and right of it (hi[d] = point M+d).
template <typename F, int M, int S>
__device__ __forceinline__ void lane_multistep_with(const F (&u)[M], F (&v)[M],
                                                    const StepWeights<F>& sw, const F (&lo)[S],
                                                    const F (&hi)[S]) {
  auto at = [&](int i) -> F { return i < 0 ? lo[-1 - i] : (i < M ? u[i] : hi[i - M]); };
#pragma unroll
  for (int j = 0; j < M; ++j) {
    F acc = sw.w[S] * (at(j - S) + at(j + S));
#pragma unroll
    for (int d = S - 1; d >= 1; --d) acc = fma_of(sw.w[d], at(j - d) + at(j + d), acc);
    v[j] = fma_of(sw.w[0], u[j], acc);
  }
}

template <typename F, int M, int S>
__device__ __forceinline__ void lane_multistep(const F (&u)[M], F (&v)[M],
                                               const StepWeights<F>& sw) {
  static_assert(S >= 2 && S <= 4 && S <= M, "fused depth");
  F lo[S], hi[S];
#pragma unroll
  for (int d = 0; d < S; ++d) {
    lo[d] = from_lower_lane(u[M - 1 - d]);  // point -1-d
    hi[d] = from_upper_lane(u[d]);          // point M+d
    // keep each neighbour value in a register of its own: left to itself the
    // compiler folds the lane shift into every addition that uses the value,
    // and a sweep full of DPP additions issues far below the VALU rate
    asm volatile("" : "+v"(lo[d]), "+v"(hi[d]));
  }
  lane_multistep_with<F, M, S>(u, v, sw, lo, hi);
}

// `steps` steps of a tile holding no rod end: pairs of fused sweeps
// (u -> v -> u), then single steps for the remainder.
template <typename F, int M, int S>
__device__ __forceinline__ void advance_interior(F (&u)[M], int steps, F r,
                                                 const StepWeights<F>& sw) {
  int s = 0;
  if constexpr (S > 1) {
    // weights in vector registers: a VALU instruction with a scalar operand
    // issues at half rate when such instructions come back to back
    StepWeights<F> vw = sw;
#pragma unroll
    for (int d = 0; d <= S; ++d) asm volatile("" : "+v"(vw.w[d]));
    F v[M];
    for (; s + 2 * S <= steps; s += 2 * S) {
      lane_multistep<F, M, S>(u, v, vw);
      lane_multistep<F, M, S>(v, u, vw);
    }
  }
  for (; s < steps; ++s) {
    const F left = from_lower_lane(u[M - 1]);
    const F right = from_upper_lane(u[0]);
    lane_step<F, M>(u, left, right, r);
  }
}

// ---------------------------------------------------------------------------
// Tile t of a rod covers rod points [t*Wout, t*Wout + L).  Tile 0 starts at
// point 0 (nothing left of the fixed end is needed) and writes [0, L-H); an
// inner tile writes [t*Wout + H, t*Wout + L - H); the last tile reaches past
// point N-1 and writes up to N.  Point N-1 is pinned to cN after every step, so
// whatever lies beyond it never reaches the interior.
//
// tile_pass: the lane's M points of tile t (already loaded into u) advance
// `steps` steps; the exact part is stored to the rod at dst.
template <typename F, int M, int S>
__device__ __forceinline__ void tile_pass(F (&u)[M], F* __restrict__ dst, int64_t N, int64_t t,
                                          int64_t tiles_per_rod, int H, int steps, F r, F c1,
                                          F cN, const StepWeights<F>& sw, bool aligned,
                                          int lane) {
  constexpr int L = kWave * M;
  const int Wout = L - 2 * H;
  const int64_t base = t * Wout;
  const int q0 = lane * M;
  const bool left_end = (t == 0);
  const int64_t qN64 = N - 1 - base;
  const bool right_end = qN64 < L;
  const int lo = left_end ? 0 : H;
  const int hi = (t == tiles_per_rod - 1) ? (int)(N - base) : (L - H);
  // Each branch stores its own registers: no merge of the two loops' states.
  if (left_end || right_end) {
    // the (at most two) tiles holding a rod end re-impose it after every step
    const int qN = right_end ? (int)qN64 : 0;
    const int lN = (qN / M);
    const int jN = uniform(qN % M);
    if (left_end) u[0] = (lane == 0) ? c1 : u[0];
    if (right_end) set_point<F, M>(u, jN, lane == lN, cN);
    for (int s = 0; s < steps; ++s) {
      const F left = from_lower_lane(u[M - 1]);
      const F right = from_upper_lane(u[0]);
      lane_step<F, M>(u, left, right, r);
      if (left_end) u[0] = (lane == 0) ? c1 : u[0];
      if (right_end) set_point<F, M>(u, jN, lane == lN, cN);
    }
    store_points<F, M>(u, dst, base + q0, q0, lo, hi, aligned);
  } else {
    advance_interior<F, M, S>(u, steps, r, sw);
    store_points<F, M>(u, dst, base + q0, q0, lo, hi, aligned);
  }
}

}  // namespace heat1d
