// kernels_adjoint.hip -- discrete adjoint of the synchronous iteration.
//
// For a loss L(u(K)) the adjoint state lambda(k) = dL/du(k) obeys
// lambda(k) = A^T lambda(k+1), where A is one step of Eq.3.  The interior block
// of A is symmetric and the ends are fixed, so A^T is the same three-point
// stencil with both ends held at zero.  The sensitivity to r collects
// lambda_i(k+1) (u_{i+1}(k) - 2u_i(k) + u_{i-1}(k)) over all steps and interior
// points, which needs the forward states in reverse order.
//
// Checkpointing, two levels:
//  * the forward pass keeps every S-th state in HBM (S = ceil(sqrt K) by
//    default);
//  * before the backward sweep crosses the stretch [jS, (j+1)S), the states at
//    the starts of its sub-stretches of S2 = 16 steps are recomputed into a
//    small HBM buffer (depth-S2 tiled passes);
//  * stretch_kernel handles one sub-stretch per launch: every wavefront loads
//    its tile of the sub-stretch's first state, recomputes the S2 - 1 states
//    that follow into registers (S2 x M values per lane, no HBM traffic),
//    then walks the S2 steps backwards with lambda in registers, pairing
//    lambda(k+1) with the register copy of u(k).
// HBM traffic is thus about five states per sub-stretch instead of two per
// step.  Each tile sums the dL/dr terms of the points it owns only (no double
// counting across overlapping halos) into a per-tile double; the partial sums
// are reduced in a fixed order, so dL/dr is deterministic.
#include "heat1d_device.h"
#include "heat1d_launch.h"

namespace heat1d {

constexpr int kSub = 16;  // steps per register-resident sub-stretch

// Deterministic wavefront sum (fixed butterfly order).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Tile t of a rod covers [t*Wout, t*Wout + L); geometry as the tiled forward
// kernel, with the halo H >= kSub + 1 so that both the recomputed states (one
// point of neighbour needed for the Laplacian) and lambda stay exact on the
// owned points for a whole sub-stretch.
template <typename F, int M>
__global__ __launch_bounds__(256) void stretch_kernel(const F* __restrict__ u_start,
                                                     const F* __restrict__ lam_in,
                                                     F* __restrict__ lam_out, int64_t N,
                                                     int64_t total_tiles, int64_t tiles_per_rod,
                                                     int H, int len, F r, F c1, F cN,
                                                     double* __restrict__ partials, int aligned) {
  constexpr int L = kWave * M;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wid = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
  if (wid >= total_tiles) return;
  const int64_t rod = wid / tiles_per_rod;
  const int64_t t = wid - rod * tiles_per_rod;
  const int Wout = L - 2 * H;
  const int64_t base = t * Wout;
  const int q0 = lane * M;

  const bool left_end = (t == 0);
  const int64_t qN64 = N - 1 - base;
  const bool right_end = qN64 < L;
  const int qN = right_end ? (int)qN64 : 0;
  const int lN = qN / M;
  const int jN = uniform(qN % M);

  // forward: u(k0 + s) for s < len, in registers
  F st[kSub][M];
  load_points<F, M>(st[0], u_start + rod * N, base + q0, N, aligned != 0);
  if (left_end) st[0][0] = (lane == 0) ? c1 : st[0][0];
  if (right_end) set_point_select<F, M>(st[0], jN, lane == lN, cN);
#pragma unroll
  for (int s = 1; s < kSub; ++s) {
    if (s < len) {
      const F left = from_lower_lane(st[s - 1][M - 1]);
      const F right = from_upper_lane(st[s - 1][0]);
      F prev = left;
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const F nx = (j + 1 < M) ? st[s - 1][j + 1] : right;
        st[s][j] = eq3_step(prev, st[s - 1][j], nx, r);
        prev = st[s - 1][j];
      }
      if (left_end) st[s][0] = (lane == 0) ? c1 : st[s][0];
      if (right_end) set_point_select<F, M>(st[s], jN, lane == lN, cN);
    }
  }

  // backward: lambda(k0 + len) -> lambda(k0)
  F lam[M];
  load_points<F, M>(lam, lam_in + rod * N, base + q0, N, aligned != 0);
  if (left_end) lam[0] = (lane == 0) ? F(0) : lam[0];
  if (right_end) set_point_select<F, M>(lam, jN, lane == lN, F(0));

  // points whose dL/dr terms this tile owns: its output range, interior only
  const int lo = left_end ? 1 : H;
  const int hi = (t == tiles_per_rod - 1) ? (int)(N - 1 - base) : (L - H);
  double acc = 0.0;
#pragma unroll
  for (int s = kSub - 1; s >= 0; --s) {
    if (s < len) {
      // dL/dr term: lambda(k0+s+1) . Laplacian of u(k0+s)
      const F ul = from_lower_lane(st[s][M - 1]);
      const F ur = from_upper_lane(st[s][0]);
      F part = F(0);
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const F a = (j == 0) ? ul : st[s][j - 1];
        const F b = (j + 1 < M) ? st[s][j + 1] : ur;
        const F lap = fma_of(F(-2), st[s][j], a + b);
        const int q = q0 + j;
        part += (q >= lo && q < hi) ? lam[j] * lap : F(0);
      }
      acc += (double)part;
      // lambda(k0+s) = A^T lambda(k0+s+1)
      const F left = from_lower_lane(lam[M - 1]);
      const F right = from_upper_lane(lam[0]);
      lane_step<F, M>(lam, left, right, r);
      if (left_end) lam[0] = (lane == 0) ? F(0) : lam[0];
      if (right_end) set_point_select<F, M>(lam, jN, lane == lN, F(0));
    }
  }
  const int olo = left_end ? 0 : H;
  const int ohi = (t == tiles_per_rod - 1) ? (int)(N - base) : (L - H);
  store_points<F, M>(lam, lam_out + rod * N, base + q0, q0, olo, ohi, aligned != 0);
  const double tot = wave_sum(acc);
  if (lane == 0) partials[wid] = tot;
}

// grad_r[b] = sum over g < nseg, t < tiles of partials[(g*nrods + b)*tiles + t].
// One workgroup per rod; thread i sums the entries i, i+256, ... in order, then
// a fixed LDS tree combines the 256 sums: the same order on every run.
__global__ __launch_bounds__(256) void reduce_partials_kernel(const double* __restrict__ partials,
                                                              int64_t nseg, int64_t nrods,
                                                              int64_t tiles_per_rod,
                                                              double* __restrict__ grad_r) {
  __shared__ double sh[256];
  const int64_t b = blockIdx.x;
  const int64_t n = nseg * tiles_per_rod;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const int64_t g = i / tiles_per_rod;
    const int64_t t = i - g * tiles_per_rod;
    acc += partials[(g * nrods + b) * tiles_per_rod + t];
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) grad_r[b] = sh[0];
}

// ---------------------------------------------------------------------------
static bool is_aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

int stretch_steps() { return kSub; }

int stretch_pts_per_lane(int dtype) { return dtype == 0 ? 8 : 4; }

TileGeom stretch_geometry(int dtype, int64_t N) {
  return tile_geometry(dtype, stretch_pts_per_lane(dtype), kSub + 1, N);
}

template <typename F, int M>
static void stretch_launch(const TileGeom& g, const void* u_start, const void* lam_in,
                           void* lam_out, int64_t N, int64_t nrods, int len, double r, double c1,
                           double cN, double* partials, hipStream_t s) {
  const int64_t total = g.tiles_per_rod * nrods;
  const int64_t blocks = (total + 3) / 4;
  const int V = Vec<F>::n;
  const int aligned = is_aligned16(u_start) && is_aligned16(lam_in) && is_aligned16(lam_out) &&
                      (nrods == 1 || N % V == 0);
  hipLaunchKernelGGL((stretch_kernel<F, M>), dim3((unsigned)blocks), dim3(256), 0, s,
                     (const F*)u_start, (const F*)lam_in, (F*)lam_out, N, total, g.tiles_per_rod,
                     g.H, len, (F)r, (F)c1, (F)cN, partials, aligned);
}

hipError_t launch_adjoint_stretch(int dtype, const TileGeom& g, const void* u_start,
                                  const void* lam_in, void* lam_out, int64_t N, int64_t nrods,
                                  int len, double r, double c1, double cN, double* partials,
                                  hipStream_t s) {
  if (len < 1 || len > kSub || g.H < kSub + 1 || g.tiles_per_rod <= 0) return hipErrorInvalidValue;
  if (g.M != stretch_pts_per_lane(dtype)) return hipErrorInvalidValue;
  if (dtype == 0)
    stretch_launch<float, 8>(g, u_start, lam_in, lam_out, N, nrods, len, r, c1, cN, partials, s);
  else
    stretch_launch<double, 4>(g, u_start, lam_in, lam_out, N, nrods, len, r, c1, cN, partials, s);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const double* partials, int64_t nseg, int64_t nrods,
                                  int64_t tiles_per_rod, double* grad_r, hipStream_t s) {
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)(nrods > 0 ? nrods : 1)), dim3(256), 0,
                     s, partials, nseg, nrods, tiles_per_rod, grad_r);
  return hipGetLastError();
}

}  // namespace heat1d
