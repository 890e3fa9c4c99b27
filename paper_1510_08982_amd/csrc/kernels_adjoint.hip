// kernels_adjoint.hip -- discrete adjoint of the synchronous iteration.
//
// For a loss L(u(K)) the adjoint state lambda(k) = dL/du(k) obeys
// lambda(k) = A^T lambda(k+1), where A is one step of Eq.3.  The interior block
// of A is symmetric and the ends are fixed, so A^T is the same three-point
// stencil with both ends held at zero.  The sensitivity to r collects
// lambda_i(k+1) (u_{i+1}(k) - 2u_i(k) + u_{i-1}(k)) over all steps and interior
// points, which needs the forward states in reverse order: the forward pass
// keeps every S-th state (checkpoints), and each stretch of S steps is
// recomputed just before the backward sweep crosses it.
//
//  record_kernel  recompute one stretch from its checkpoint with the depth-T
//                 tile scheme, writing every intermediate state.
//  sweep_kernel   tile-wise backward sweep over one stretch: lambda stays in
//                 registers, u(k) is read per step for the dL/dr term, and each
//                 tile sums its own points only (no double counting across the
//                 overlapping halos).  Per-tile sums go to a partials array and
//                 are reduced in a fixed order, so dL/dr is deterministic.
#include "heat1d_device.h"
#include "heat1d_launch.h"

namespace heat1d {

template <typename F, int M>
__global__ __launch_bounds__(256) void record_kernel(const F* __restrict__ in,
                                                     F* __restrict__ states, int64_t stride,
                                                     int64_t N, int64_t total_tiles,
                                                     int64_t tiles_per_rod, int H, int nsteps,
                                                     F r, F c1, F cN, int aligned) {
  constexpr int L = kWave * M;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wid = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
  if (wid >= total_tiles) return;
  const int64_t rod = wid / tiles_per_rod;
  const int64_t t = wid - rod * tiles_per_rod;
  const int Wout = L - 2 * H;
  const int64_t base = t * Wout;
  const F* __restrict__ src = in + rod * N;

  F u[M];
  const int q0 = lane * M;
  load_points<F, M>(u, src, base + q0, N, aligned != 0);
  const bool left_end = (t == 0);
  const int64_t qN64 = N - 1 - base;
  const bool right_end = qN64 < L;
  const int qN = right_end ? (int)qN64 : 0;
  const int lN = qN / M;
  const int jN = uniform(qN % M);
  if (left_end) u[0] = (lane == 0) ? c1 : u[0];
  if (right_end) set_point<F, M>(u, jN, lane == lN, cN);
  const int lo = left_end ? 0 : H;
  const int hi = (t == tiles_per_rod - 1) ? (int)(N - base) : (L - H);

  for (int s = 0; s < nsteps; ++s) {
    const F left = from_lower_lane(u[M - 1]);
    const F right = from_upper_lane(u[0]);
    lane_step<F, M>(u, left, right, r);
    if (left_end) u[0] = (lane == 0) ? c1 : u[0];
    if (right_end) set_point<F, M>(u, jN, lane == lN, cN);
    F* dst = states + (int64_t)s * stride + rod * N;
    store_points<F, M>(u, dst, base + q0, q0, lo, hi, aligned != 0);
  }
}

// Deterministic wavefront sum (fixed butterfly order).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

template <typename F, int M>
__global__ __launch_bounds__(256) void sweep_kernel(const F* __restrict__ lam_in,
                                                    F* __restrict__ lam_out,
                                                    const F* __restrict__ u_first,
                                                    const F* __restrict__ states, int64_t stride,
                                                    int64_t N, int64_t total_tiles,
                                                    int64_t tiles_per_rod, int H, int len, F r,
                                                    double* __restrict__ partials, int aligned) {
  constexpr int L = kWave * M;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wid = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
  if (wid >= total_tiles) return;
  const int64_t rod = wid / tiles_per_rod;
  const int64_t t = wid - rod * tiles_per_rod;
  const int Wout = L - 2 * H;
  const int64_t base = t * Wout;

  F lam[M];
  const int q0 = lane * M;
  load_points<F, M>(lam, lam_in + rod * N, base + q0, N, aligned != 0);
  const bool left_end = (t == 0);
  const int64_t qN64 = N - 1 - base;
  const bool right_end = qN64 < L;
  const int qN = right_end ? (int)qN64 : 0;
  const int lN = qN / M;
  const int jN = uniform(qN % M);
  // lambda vanishes at the fixed ends
  if (left_end) lam[0] = (lane == 0) ? F(0) : lam[0];
  if (right_end) set_point<F, M>(lam, jN, lane == lN, F(0));

  // points of this tile whose dL/dr terms this tile owns: its output range,
  // restricted to the interior 1..N-2
  const int lo = left_end ? 1 : H;
  const int hi = (t == tiles_per_rod - 1) ? (int)(N - 1 - base) : (L - H);

  double acc = 0.0;
  for (int s = 0; s < len; ++s) {
    const int i = len - 1 - s;  // u(k0 + i) pairs with lambda(k0 + i + 1)
    const F* __restrict__ us = (i == 0 ? u_first : states + (int64_t)(i - 1) * stride) + rod * N;
    F u[M];
    load_points<F, M>(u, us, base + q0, N, aligned != 0);
    const F ul = from_lower_lane(u[M - 1]);
    const F ur = from_upper_lane(u[0]);
    F part = F(0);
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const F a = (j == 0) ? ul : u[j - 1];
      const F b = (j + 1 < M) ? u[j + 1] : ur;
      const F lap = __builtin_fma(F(-2), u[j], a + b);
      const int q = q0 + j;
      const F term = (q >= lo && q < hi) ? lam[j] * lap : F(0);
      part += term;
    }
    acc += (double)part;
    const F left = from_lower_lane(lam[M - 1]);
    const F right = from_upper_lane(lam[0]);
    lane_step<F, M>(lam, left, right, r);
    if (left_end) lam[0] = (lane == 0) ? F(0) : lam[0];
    if (right_end) set_point<F, M>(lam, jN, lane == lN, F(0));
  }
  const int olo = left_end ? 0 : H;
  const int ohi = (t == tiles_per_rod - 1) ? (int)(N - base) : (L - H);
  store_points<F, M>(lam, lam_out + rod * N, base + q0, q0, olo, ohi, aligned != 0);
  const double tot = wave_sum(acc);
  if (lane == 0) partials[wid] = tot;
}

__global__ void reduce_partials_kernel(const double* __restrict__ partials, int64_t nseg,
                                       int64_t nrods, int64_t tiles_per_rod,
                                       double* __restrict__ grad_r) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nrods) return;
  double s = 0.0;
  for (int64_t g = 0; g < nseg; ++g)
    for (int64_t t = 0; t < tiles_per_rod; ++t)
      s += partials[(g * nrods + b) * tiles_per_rod + t];
  grad_r[b] = s;
}

// ---------------------------------------------------------------------------
static bool is_aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

template <typename F, int M>
static void record_launch(const TileGeom& g, const void* in, void* states, int64_t stride,
                          int64_t N, int64_t nrods, int len, double r, double c1, double cN,
                          hipStream_t s) {
  const int64_t total = g.tiles_per_rod * nrods;
  const int64_t blocks = (total + 3) / 4;
  const int V = Vec<F>::n;
  const int aligned = is_aligned16(in) && is_aligned16(states) && (nrods == 1 || N % V == 0) &&
                      (stride % V == 0);
  hipLaunchKernelGGL((record_kernel<F, M>), dim3((unsigned)blocks), dim3(256), 0, s,
                     (const F*)in, (F*)states, stride, N, total, g.tiles_per_rod, g.H, len - 1,
                     (F)r, (F)c1, (F)cN, aligned);
}

template <typename F, int M>
static void sweep_launch(const TileGeom& g, const void* lam_in, void* lam_out, const void* u_first,
                         const void* states, int64_t stride, int64_t N, int64_t nrods, int len,
                         double r, double* partials, hipStream_t s) {
  const int64_t total = g.tiles_per_rod * nrods;
  const int64_t blocks = (total + 3) / 4;
  const int V = Vec<F>::n;
  const int aligned = is_aligned16(lam_in) && is_aligned16(lam_out) && is_aligned16(u_first) &&
                      is_aligned16(states) && (nrods == 1 || N % V == 0) && (stride % V == 0);
  hipLaunchKernelGGL((sweep_kernel<F, M>), dim3((unsigned)blocks), dim3(256), 0, s,
                     (const F*)lam_in, (F*)lam_out, (const F*)u_first, (const F*)states, stride, N,
                     total, g.tiles_per_rod, g.H, len, (F)r, partials, aligned);
}

hipError_t launch_record(int dtype, const TileGeom& g, const void* in, void* states,
                         int64_t stride, int64_t N, int64_t nrods, int len, double r, double c1,
                         double cN, hipStream_t s) {
  if (len - 1 > g.H || g.tiles_per_rod <= 0) return hipErrorInvalidValue;
  if (len <= 1) return hipSuccess;
#define HEAT1D_REC(FT, MM)                                                        \
  case MM:                                                                        \
    record_launch<FT, MM>(g, in, states, stride, N, nrods, len, r, c1, cN, s);    \
    break;
  if (dtype == 0) {
    switch (g.M) {
      HEAT1D_REC(float, 16)
      HEAT1D_REC(float, 32)
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (g.M) {
      HEAT1D_REC(double, 16)
      HEAT1D_REC(double, 32)
      default: return hipErrorInvalidValue;
    }
  }
#undef HEAT1D_REC
  return hipGetLastError();
}

hipError_t launch_adjoint_sweep(int dtype, const TileGeom& g, const void* lam_in, void* lam_out,
                                const void* u_first, const void* states, int64_t stride,
                                int64_t N, int64_t nrods, int len, double r, double* partials,
                                hipStream_t s) {
  if (len > g.H || g.tiles_per_rod <= 0) return hipErrorInvalidValue;
#define HEAT1D_SW(FT, MM)                                                                  \
  case MM:                                                                                 \
    sweep_launch<FT, MM>(g, lam_in, lam_out, u_first, states, stride, N, nrods, len, r,    \
                         partials, s);                                                     \
    break;
  if (dtype == 0) {
    switch (g.M) {
      HEAT1D_SW(float, 16)
      HEAT1D_SW(float, 32)
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (g.M) {
      HEAT1D_SW(double, 16)
      HEAT1D_SW(double, 32)
      default: return hipErrorInvalidValue;
    }
  }
#undef HEAT1D_SW
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const double* partials, int64_t nseg, int64_t nrods,
                                  int64_t tiles_per_rod, double* grad_r, hipStream_t s) {
  const int64_t blocks = (nrods + 63) / 64;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)blocks), dim3(64), 0, s, partials,
                     nseg, nrods, tiles_per_rod, grad_r);
  return hipGetLastError();
}

}  // namespace heat1d
