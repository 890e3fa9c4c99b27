// heat1d_steps.h -- register sweeps shared by the tiled, pipelined and
// dataflow synchronous kernels: fused S-step sweeps and the host-side weights
// of the S-step stencil.
#pragma once

#include "heat1d_device.h"

namespace heat1d {

// Fused steps.  S steps of Eq.3 on points away from the rod ends equal one
// application of the S-step stencil u_i <- w_0 u_i + sum_{d=1..S} w_d
// (u_{i-d} + u_{i+d}), whose weights are the coefficients of the S-th power of
// the three-point stencil (r, 1-2r, r) (all positive for r <= 1/2).  Per point
// that is S additions, one multiplication and S fused multiply-adds, 2 + 1/S
// instructions per point update instead of 3, with fewer roundings.  The
// garbage entering a tile at its two cut edges still advances one point per
// step, so the halo rule H >= steps is unchanged.
template <typename F>
struct StepWeights {
  F w[5];  // w[0..S]
};

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
// Agent-coherent access to a state that other CUs (on other XCDs, whose L2
// caches are not coherent with this one) write during the same launch: 64-bit
// relaxed atomics at agent scope, two FP32 points or one FP64 point per word.
// Rods, tile starts and per-lane runs are whole words (N even).
template <typename F> struct WordPts;
template <> struct WordPts<float> { static constexpr int n = 2; };
template <> struct WordPts<double> { static constexpr int n = 1; };

template <typename F, int M>
__device__ __forceinline__ uint64_t coherent_word(const F* p) {
  return __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

template <typename F, int P>
__device__ __forceinline__ void unpack_word(uint64_t w, F* out) {
  if constexpr (P == 2) {
    out[0] = __uint_as_float((uint32_t)w);
    out[1] = __uint_as_float((uint32_t)(w >> 32));
  } else {
    out[0] = __longlong_as_double((long long)w);
  }
}

template <typename F, int M>
__device__ __forceinline__ void load_coherent(F (&u)[M], const F* __restrict__ src, int64_t g0,
                                              int64_t n) {
  constexpr int P = WordPts<F>::n;
  static_assert(M % P == 0, "whole words per lane");
  const F* p = src + g0;
  if (g0 + M <= n) {
    // the common case: one base address, constant offsets
#pragma unroll
    for (int c = 0; c < M / P; ++c) unpack_word<F, P>(coherent_word<F, M>(p + c * P), &u[c * P]);
  } else {
    // a lane at or past the rod's end: words past n are not read (their
    // points lie beyond the pinned end and are never stored)
    int64_t left = n - g0;
    asm volatile("" : "+v"(left));
#pragma unroll
    for (int c = 0; c < M / P; ++c) {
      uint64_t w = 0;
      if (c * P < left) w = coherent_word<F, M>(p + c * P);
      unpack_word<F, P>(w, &u[c * P]);
    }
  }
}

// Store the lane's points whose local index q0+j lies in [lo, hi) at rod index
// g0+j (lo, hi even for FP32, so words are never split).  The range goes
// through an empty asm so that the per-word tests stay here: hoisted out of a
// persistent kernel's tile loop they would hold a mask register pair each for
// the whole kernel.
template <typename F, int M>
__device__ __forceinline__ void store_coherent(const F (&u)[M], F* __restrict__ dst, int64_t g0,
                                               int q0, int lo, int hi) {
  constexpr int P = WordPts<F>::n;
  asm volatile("" : "+v"(lo), "+v"(hi), "+v"(q0));
  F* p = dst + g0;
  const bool whole = q0 >= lo && q0 + M <= hi;
#pragma unroll
  for (int c = 0; c < M / P; ++c) {
    const int q = q0 + c * P;
    if (whole || (q >= lo && q + P <= hi)) {
      uint64_t w;
      if constexpr (P == 2)
        w = (uint64_t)__float_as_uint(u[2 * c]) | ((uint64_t)__float_as_uint(u[2 * c + 1]) << 32);
      else
        w = (uint64_t)__double_as_longlong(u[c]);
      __hip_atomic_store(reinterpret_cast<uint64_t*>(p + c * P), w, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
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
// `steps` steps; the exact part is stored to the rod at dst, with plain
// stores or, kCoherent, with agent-coherent 64-bit stores.
template <typename F, int M, int S, bool kCoherent>
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
    if constexpr (kCoherent)
      store_coherent<F, M>(u, dst, base + q0, q0, lo, hi);
    else
      store_points<F, M>(u, dst, base + q0, q0, lo, hi, aligned);
  } else {
    advance_interior<F, M, S>(u, steps, r, sw);
    if constexpr (kCoherent)
      store_coherent<F, M>(u, dst, base + q0, q0, lo, hi);
    else
      store_points<F, M>(u, dst, base + q0, q0, lo, hi, aligned);
  }
}

// Weights of the S-step stencil: coefficients of (r, 1-2r, r)^S, in double.
template <typename F>
inline StepWeights<F> step_weights(double r, int S) {
  double c[9] = {1.0, 0, 0, 0, 0, 0, 0, 0, 0};  // polynomial in x, centre at index S
  int len = 1;
  for (int k = 0; k < S; ++k) {
    double n[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = 0; i < len; ++i) {
      n[i] += r * c[i];
      n[i + 1] += (1.0 - 2.0 * r) * c[i];
      n[i + 2] += r * c[i];
    }
    len += 2;
    for (int i = 0; i < len; ++i) c[i] = n[i];
  }
  StepWeights<F> w{};
  for (int d = 0; d <= S && d < 5; ++d) w.w[d] = (F)c[S + d];
  return w;
}

}  // namespace heat1d
