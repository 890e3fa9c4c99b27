// heat1d_device.h -- device-side building blocks shared by the gfx950 kernels.
//
// Register layout used by every kernel: a wavefront holds 64*M consecutive
// points, lane l holding points [l*M, l*M + M) of its tile in registers u[0..M).
// One time step needs, per lane, the last point of the lane below and the first
// point of the lane above; both arrive through DPP wavefront shifts, so a step
// costs three VALU instructions per point plus two lane moves per lane.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace heat1d {

constexpr int kWave = 64;

// One step of Eq.3 (Section 2).  Written as c + r((a+b) - 2c): algebraically
// r a + (1-2r) c + r b, but a constant state stays exactly constant and no
// coefficient (1-2r) has to be rounded.  a is the left neighbour, b the right
// one; a+b is commutative, so mirrored inputs give mirrored bits.
__device__ __forceinline__ float eq3_step(float a, float c, float b, float r) {
  return __builtin_fmaf(r, __builtin_fmaf(-2.0f, c, a + b), c);
}
__device__ __forceinline__ double eq3_step(double a, double c, double b, double r) {
  return __builtin_fma(r, __builtin_fma(-2.0, c, a + b), c);
}

// Fused multiply-add in the precision of the operands (a*b + c, one rounding).
__device__ __forceinline__ float fma_of(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_of(double a, double b, double c) { return __builtin_fma(a, b, c); }

// DPP control words of the gfx9 wavefront shifts.
constexpr int kDppWaveShr1 = 0x138;  // lane i reads lane i-1
constexpr int kDppWaveShl1 = 0x130;  // lane i reads lane i+1

template <int Ctrl>
__device__ __forceinline__ int dpp_i32(int x) {
  return __builtin_amdgcn_update_dpp(0, x, Ctrl, 0xF, 0xF, true);
}
template <int Ctrl>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(dpp_i32<Ctrl>(__float_as_int(x)));
}
template <int Ctrl>
__device__ __forceinline__ double dpp(double x) {
  const int lo = dpp_i32<Ctrl>(__double2loint(x));
  const int hi = dpp_i32<Ctrl>(__double2hiint(x));
  return __hiloint2double(hi, lo);
}
// Value held by lane-1 (lane 0 gets 0).
template <typename F>
__device__ __forceinline__ F from_lower_lane(F x) { return dpp<kDppWaveShr1>(x); }
// Value held by lane+1 (lane 63 gets 0).
template <typename F>
__device__ __forceinline__ F from_upper_lane(F x) { return dpp<kDppWaveShl1>(x); }

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ float read_lane(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ double read_lane(double x, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
  return __hiloint2double(hi, lo);
}

// Advance one lane's M points by one step.  left/right are the neighbours of
// u[0] and u[M-1].
template <typename F, int M>
__device__ __forceinline__ void lane_step(F (&u)[M], F left, F right, F r) {
  F prev = left;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const F c = u[j];
    const F nx = (j + 1 < M) ? u[j + 1] : right;
    u[j] = eq3_step(prev, c, nx, r);
    prev = c;
  }
}

// Write v into register j (a wave-uniform index) of the lanes where `mine`
// holds.  Up to 128 bytes of points per lane the compiler indexes the register
// file directly (gpr-index mode: a few instructions).  Larger arrays would be
// demoted to scratch memory that way, so they use one select per register
// with a scalar condition instead (about M vector and 3M scalar
// instructions); only the wavefront holding the pinned point executes it.
// The select form alone, for arrays that are rows of a larger register array
// (indexing such a row would demote the whole array to scratch memory).
template <typename F, int M>
__device__ __forceinline__ void set_point_select(F (&u)[M], int j, bool mine, F v) {
  int jl = j;
  asm volatile("" : "+s"(jl));
#pragma unroll
  for (int jj = 0; jj < M; ++jj) u[jj] = (mine && jj == jl) ? v : u[jj];
}

template <typename F, int M>
__device__ __forceinline__ void set_point(F (&u)[M], int j, bool mine, F v) {
  if constexpr (M * sizeof(F) <= 128) {
    const int ju = uniform(j);
    const F cur = u[ju];
    u[ju] = mine ? v : cur;
  } else {
    // the select form; the asm re-materialises the index next to its use so
    // that the M scalar conditions are not hoisted (and spilled) out of loops
    set_point_select<F, M>(u, j, mine, v);
  }
}
// Register j (wave-uniform index) of every lane, found by a binary search of
// scalar branches on j; the empty volatile asm in each leaf keeps the compiler
// from turning the search into M selects.
template <typename F, int M, int LO = 0, int HI = M>
__device__ __forceinline__ F get_point(const F (&u)[M], int j) {
  if constexpr (HI - LO == 1) {
    F x = u[LO];
    asm volatile("" : "+v"(x));
    return x;
  } else {
    constexpr int MID = (LO + HI) / 2;
    if (j < MID) return get_point<F, M, LO, MID>(u, j);
    return get_point<F, M, MID, HI>(u, j);
  }
}

// Vector type of 16 bytes for coalesced loads / stores.
template <typename F> struct Vec;
template <> struct Vec<float> { using T = float4; static constexpr int n = 4; };
template <> struct Vec<double> { using T = double2; static constexpr int n = 2; };

// Load lane's M points starting at rod index g0 (may be negative or run past
// n); points outside [0, n) read as 0.  `aligned` says that src + g0 is 16-byte
// aligned whenever g0 is a multiple of the vector width.  Bounds are turned
// into a 32-bit register range [jlo, jhi) once, so no 64-bit index per point
// stays live.
template <typename F, int M>
__device__ __forceinline__ void load_points(F (&u)[M], const F* __restrict__ src, int64_t g0,
                                            int64_t n, bool aligned) {
  constexpr int V = Vec<F>::n;
  using VT = typename Vec<F>::T;
  const F* __restrict__ p = src + g0;
  const int jlo = g0 >= 0 ? 0 : (-g0 >= M ? M : (int)(-g0));
  const int64_t left = n - g0;
  const int jhi = left >= M ? M : (left <= 0 ? 0 : (int)left);
  if ((M % V) == 0 && aligned && jlo == 0 && jhi == M) {
#pragma unroll
    for (int c = 0; c < M / V; ++c) {
      const VT v = *reinterpret_cast<const VT*>(p + c * V);
      const F* pv = reinterpret_cast<const F*>(&v);
#pragma unroll
      for (int e = 0; e < V; ++e) u[c * V + e] = pv[e];
    }
  } else {
#pragma unroll
    for (int j = 0; j < M; ++j) u[j] = (j >= jlo && j < jhi) ? p[j] : F(0);
  }
}

// Whole-vector load of the lane's M points starting at rod index g0, for rods
// whose length n and tile starts are multiples of the vector width and whose
// storage is 16-byte aligned.  A vector at or past n (only in the last tile of
// a rod, beyond the pinned point n-1) reads the rod's first vector instead:
// those registers are never stored and never reach a point below n-1, because
// n-1 is re-pinned after every step.  One load path and no select on the
// loaded values, so a prefetch into these registers needs no wait until the
// values are used.
template <typename F, int M>
__device__ __forceinline__ void load_points_vec(F (&u)[M], const F* __restrict__ src, int64_t g0,
                                                int64_t n) {
  constexpr int V = Vec<F>::n;
  using VT = typename Vec<F>::T;
  static_assert(M % V == 0, "whole vectors per lane");
#pragma unroll
  for (int c = 0; c < M / V; ++c) {
    const int64_t gc = g0 + c * V;
    const VT v = *reinterpret_cast<const VT*>(src + (gc < n ? gc : 0));
    const F* pv = reinterpret_cast<const F*>(&v);
#pragma unroll
    for (int e = 0; e < V; ++e) u[c * V + e] = pv[e];
  }
}

// Store the lane's points whose local index q0+j lies in [lo, hi) to dst at
// rod index g0+j.
template <typename F, int M>
__device__ __forceinline__ void store_points(const F (&u)[M], F* __restrict__ dst, int64_t g0,
                                             int q0, int lo, int hi, bool aligned) {
  constexpr int V = Vec<F>::n;
  using VT = typename Vec<F>::T;
  F* __restrict__ p = dst + g0;
  if ((M % V) == 0 && aligned && q0 >= lo && q0 + M <= hi) {
#pragma unroll
    for (int c = 0; c < M / V; ++c) {
      VT v;
      F* pv = reinterpret_cast<F*>(&v);
#pragma unroll
      for (int e = 0; e < V; ++e) pv[e] = u[c * V + e];
      *reinterpret_cast<VT*>(p + c * V) = v;
    }
  } else if (q0 + M > lo && q0 < hi) {
    const int jlo = lo - q0, jhi = hi - q0;
#pragma unroll
    for (int j = 0; j < M; ++j)
      if (j >= jlo && j < jhi) p[j] = u[j];
  }
}

// ---------------------------------------------------------------------------
// Delay schedule of the emulated asynchronous mode.  The mixing function is the
// SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014): add the
// 64-bit golden-ratio increment, then two xor-shift-multiply rounds and a final
// xor-shift.  delta = ((x >> 32) * (d+1)) >> 32 maps the top 32 bits to 0..d.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint64_t sm64(uint64_t s) {
  uint64_t z = s + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__host__ __device__ __forceinline__ int delay_of(uint64_t seed, int64_t k, int64_t p, int side,
                                                 int64_t P, int d) {
  const uint64_t c = (((uint64_t)k * (uint64_t)P + (uint64_t)p) << 1) | (uint64_t)(side & 1);
  const uint64_t x = sm64(seed ^ sm64(c));
  return (int)(((x >> 32) * (uint64_t)(d + 1)) >> 32);
}

}  // namespace heat1d
