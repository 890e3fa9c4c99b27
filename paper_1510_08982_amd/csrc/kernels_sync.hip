// kernels_sync.hip -- synchronous iteration of Eq.3 (Section 2) on gfx950.
//
//  sync_step_kernel      one launch per step, two global buffers (the device-
//                        resident form of the paper's one-kernel-per-step loop).
//                        HBM bound: 2 elements of traffic per point update.
//  sync_tiled_kernel     depth-T temporal blocking: each wavefront loads a tile
//                        of 64*M points into registers, advances it `steps`
//                        steps with DPP lane exchange only, and writes the
//                        middle part, whose values are exact because the halo H
//                        on each side is at least `steps` deep.  Traffic per
//                        point update falls to about 2/T elements.
//  sync_resident_kernel  one workgroup holds a whole rod for all K steps.
#include "heat1d_device.h"
#include "heat1d_launch.h"
#include "heat1d_rod.h"

namespace heat1d {

// ---------------------------------------------------------------------------
template <typename F>
__global__ __launch_bounds__(256) void sync_step_kernel(const F* __restrict__ in,
                                                        F* __restrict__ out, int64_t N, F r,
                                                        F c1, F cN, int aligned) {
  constexpr int V = Vec<F>::n;
  using VT = typename Vec<F>::T;
  const int64_t rod = blockIdx.y;
  const F* __restrict__ src = in + rod * N;
  F* __restrict__ dst = out + rod * N;
  const int64_t nchunks = (N + V - 1) / V;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nchunks; c += stride) {
    const int64_t i0 = c * V;
    F v[V + 2];
    v[0] = i0 > 0 ? src[i0 - 1] : F(0);
    if (aligned && i0 + V <= N) {
      const VT x = *reinterpret_cast<const VT*>(src + i0);
      const F* px = reinterpret_cast<const F*>(&x);
#pragma unroll
      for (int e = 0; e < V; ++e) v[e + 1] = px[e];
    } else {
#pragma unroll
      for (int e = 0; e < V; ++e) v[e + 1] = (i0 + e < N) ? src[i0 + e] : F(0);
    }
    v[V + 1] = (i0 + V < N) ? src[i0 + V] : F(0);
    // the ends hold c1 / cN at every step, including in the initial state
#pragma unroll
    for (int e = 0; e < V + 2; ++e) {
      const int64_t g = i0 - 1 + e;
      v[e] = (g == 0) ? c1 : (g == N - 1) ? cN : v[e];
    }
    F o[V];
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const int64_t i = i0 + e;
      o[e] = (i == 0) ? c1 : (i == N - 1) ? cN : eq3_step(v[e], v[e + 1], v[e + 2], r);
    }
    if (aligned && i0 + V <= N) {
      VT x;
      F* px = reinterpret_cast<F*>(&x);
#pragma unroll
      for (int e = 0; e < V; ++e) px[e] = o[e];
      *reinterpret_cast<VT*>(dst + i0) = x;
    } else {
#pragma unroll
      for (int e = 0; e < V; ++e)
        if (i0 + e < N) dst[i0 + e] = o[e];
    }
  }
}

// ---------------------------------------------------------------------------
// Tile t of a rod covers rod points [t*Wout, t*Wout + L).  Tile 0 starts at
// point 0 (nothing left of the fixed end is needed) and writes [0, L-H); an
// inner tile writes [t*Wout + H, t*Wout + L - H); the last tile reaches past
// point N-1 and writes up to N.  Point N-1 is pinned to cN after every step, so
// whatever lies beyond it never reaches the interior.
template <typename F, int M>
__global__ __launch_bounds__(256) void sync_tiled_kernel(const F* __restrict__ in,
                                                         F* __restrict__ out, int64_t N,
                                                         int64_t total_tiles,
                                                         int64_t tiles_per_rod, int H, int steps,
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
  F* __restrict__ dst = out + rod * N;

  F u[M];
  const int q0 = lane * M;
  load_points<F, M>(u, src, base + q0, N, aligned != 0);

  const bool left_end = (t == 0);
  const int64_t qN64 = N - 1 - base;
  const bool right_end = qN64 < L;
  const int qN = right_end ? (int)qN64 : 0;
  const int lN = (qN / M);
  const int jN = uniform(qN % M);
  if (left_end) u[0] = (lane == 0) ? c1 : u[0];
  if (right_end) set_point<F, M>(u, jN, lane == lN, cN);

  if (left_end || right_end) {
    // the (at most two) tiles holding a rod end re-impose it after every step
    for (int s = 0; s < steps; ++s) {
      const F left = from_lower_lane(u[M - 1]);
      const F right = from_upper_lane(u[0]);
      lane_step<F, M>(u, left, right, r);
      if (left_end) u[0] = (lane == 0) ? c1 : u[0];
      if (right_end) set_point<F, M>(u, jN, lane == lN, cN);
    }
  } else {
    for (int s = 0; s < steps; ++s) {
      const F left = from_lower_lane(u[M - 1]);
      const F right = from_upper_lane(u[0]);
      lane_step<F, M>(u, left, right, r);
    }
  }

  const int lo = left_end ? 0 : H;
  const int hi = (t == tiles_per_rod - 1) ? (int)(N - base) : (L - H);
  store_points<F, M>(u, dst, base + q0, q0, lo, hi, aligned != 0);
}

// ---------------------------------------------------------------------------
template <typename F, int M>
__global__ __launch_bounds__(1024) void sync_resident_kernel(const F* __restrict__ in,
                                                             F* __restrict__ out, int64_t N,
                                                             int K, F r, F c1, F cN,
                                                             int aligned) {
  __shared__ F lds[4 * 16];
  const int nwaves = blockDim.x / kWave;
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t rod = blockIdx.x;
  rod_resident<F, M, RodSync::kWorkgroup>(in + rod * N, out + rod * N, (int)N, K, r, c1, cN, lds, nwaves, wave,
                           lane, aligned != 0);
}

template <typename F>
__global__ __launch_bounds__(256) void impose_ends_kernel(const F* __restrict__ in,
                                                          F* __restrict__ out, int64_t N,
                                                          int64_t total, F c1, F cN) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int64_t j = i % N;
    out[i] = (j == 0) ? c1 : (j == N - 1) ? cN : in[i];
  }
}

// ---------------------------------------------------------------------------
// Host launchers.

static bool is_aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

bool tiled_supports(int dtype, int M) {
  if (dtype == 0)
    return M == 4 || M == 8 || M == 16 || M == 24 || M == 32 || M == 40 || M == 48 || M == 64;
  return M == 2 || M == 4 || M == 8 || M == 12 || M == 16 || M == 20 || M == 24 || M == 32;
}

bool resident_supports(int dtype, int M) {
  if (dtype == 0) return M == 1 || M == 2 || M == 4 || M == 8 || M == 16 || M == 32 || M == 64;
  return M == 1 || M == 2 || M == 4 || M == 8 || M == 16 || M == 32;
}

TileGeom tile_geometry(int dtype, int M, int T, int64_t N) {
  const int V = dtype == 0 ? 4 : 2;
  TileGeom g;
  g.M = M;
  g.L = kWave * M;
  g.H = ((T + V - 1) / V) * V;
  if (g.H < V) g.H = V;
  g.Wout = g.L - 2 * g.H;
  if (g.Wout <= 0) {
    g.tiles_per_rod = 0;
    return g;
  }
  g.tiles_per_rod = (N <= g.L) ? 1 : 1 + (N - g.L + g.Wout - 1) / g.Wout;
  return g;
}

hipError_t launch_sync_step(int dtype, const void* in, void* out, int64_t N, int64_t nrods,
                            double r, double c1, double cN, hipStream_t s) {
  const int V = dtype == 0 ? 4 : 2;
  const int64_t nchunks = (N + V - 1) / V;
  int64_t blocks = (nchunks + 255) / 256;
  if (blocks > 65535) blocks = 65535;
  const int aligned = is_aligned16(in) && is_aligned16(out) && (nrods == 1 || N % V == 0);
  dim3 grid((unsigned)blocks, (unsigned)nrods);
  if (dtype == 0)
    hipLaunchKernelGGL(sync_step_kernel<float>, grid, dim3(256), 0, s, (const float*)in,
                       (float*)out, N, (float)r, (float)c1, (float)cN, aligned);
  else
    hipLaunchKernelGGL(sync_step_kernel<double>, grid, dim3(256), 0, s, (const double*)in,
                       (double*)out, N, r, c1, cN, aligned);
  return hipGetLastError();
}

template <typename F, int M>
static void tiled_launch(const TileGeom& g, const void* in, void* out, int64_t N, int64_t nrods,
                         int steps, double r, double c1, double cN, hipStream_t s) {
  const int64_t total = g.tiles_per_rod * nrods;
  const int wpb = 4;
  const int64_t blocks = (total + wpb - 1) / wpb;
  const int V = Vec<F>::n;
  const int aligned = is_aligned16(in) && is_aligned16(out) && (nrods == 1 || N % V == 0);
  hipLaunchKernelGGL((sync_tiled_kernel<F, M>), dim3((unsigned)blocks), dim3(wpb * kWave), 0, s,
                     (const F*)in, (F*)out, N, total, g.tiles_per_rod, g.H, steps, (F)r, (F)c1,
                     (F)cN, aligned);
}

hipError_t launch_sync_tiled(int dtype, const TileGeom& g, const void* in, void* out, int64_t N,
                             int64_t nrods, int steps, double r, double c1, double cN,
                             hipStream_t s) {
  if (steps > g.H || g.tiles_per_rod <= 0) return hipErrorInvalidValue;
#define HEAT1D_TILED(FT, MM)                                                   \
  case MM:                                                                     \
    tiled_launch<FT, MM>(g, in, out, N, nrods, steps, r, c1, cN, s);          \
    break;
  if (dtype == 0) {
    switch (g.M) {
      HEAT1D_TILED(float, 4)
      HEAT1D_TILED(float, 8)
      HEAT1D_TILED(float, 16)
      HEAT1D_TILED(float, 24)
      HEAT1D_TILED(float, 32)
      HEAT1D_TILED(float, 40)
      HEAT1D_TILED(float, 48)
      HEAT1D_TILED(float, 64)
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (g.M) {
      HEAT1D_TILED(double, 2)
      HEAT1D_TILED(double, 4)
      HEAT1D_TILED(double, 8)
      HEAT1D_TILED(double, 12)
      HEAT1D_TILED(double, 16)
      HEAT1D_TILED(double, 20)
      HEAT1D_TILED(double, 24)
      HEAT1D_TILED(double, 32)
      default: return hipErrorInvalidValue;
    }
  }
#undef HEAT1D_TILED
  return hipGetLastError();
}

template <typename F, int M>
static void resident_launch(int waves, const void* in, void* out, int64_t N, int64_t nrods,
                            int64_t K, double r, double c1, double cN, hipStream_t s) {
  const int V = Vec<F>::n;
  const int aligned = is_aligned16(in) && is_aligned16(out) && (nrods == 1 || N % V == 0);
  hipLaunchKernelGGL((sync_resident_kernel<F, M>), dim3((unsigned)nrods), dim3(waves * kWave), 0,
                     s, (const F*)in, (F*)out, N, (int)K, (F)r, (F)c1, (F)cN, aligned);
}

hipError_t launch_sync_resident(int dtype, int M, int waves, const void* in, void* out, int64_t N,
                                int64_t nrods, int64_t K, double r, double c1, double cN,
                                hipStream_t s) {
  if (waves < 1 || waves > 16 || (int64_t)waves * kWave * M < N) return hipErrorInvalidValue;
#define HEAT1D_RES(FT, MM)                                                     \
  case MM:                                                                     \
    resident_launch<FT, MM>(waves, in, out, N, nrods, K, r, c1, cN, s);       \
    break;
  if (dtype == 0) {
    switch (M) {
      HEAT1D_RES(float, 1)
      HEAT1D_RES(float, 2)
      HEAT1D_RES(float, 4)
      HEAT1D_RES(float, 8)
      HEAT1D_RES(float, 16)
      HEAT1D_RES(float, 32)
      HEAT1D_RES(float, 64)
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (M) {
      HEAT1D_RES(double, 1)
      HEAT1D_RES(double, 2)
      HEAT1D_RES(double, 4)
      HEAT1D_RES(double, 8)
      HEAT1D_RES(double, 16)
      HEAT1D_RES(double, 32)
      default: return hipErrorInvalidValue;
    }
  }
#undef HEAT1D_RES
  return hipGetLastError();
}

hipError_t launch_impose_ends(int dtype, const void* in, void* out, int64_t N, int64_t nrods,
                              double c1, double cN, hipStream_t s) {
  const int64_t total = N * nrods;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65535) blocks = 65535;
  if (dtype == 0)
    hipLaunchKernelGGL(impose_ends_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                       (const float*)in, (float*)out, N, total, (float)c1, (float)cN);
  else
    hipLaunchKernelGGL(impose_ends_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                       (const double*)in, (double*)out, N, total, c1, cN);
  return hipGetLastError();
}

}  // namespace heat1d
