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
//  sync_pipelined_kernel the same pass with persistent wavefronts that load
//                        their next tile while computing the current one.
//  sync_resident_kernel  one workgroup holds a whole rod for all K steps.
#include <algorithm>
#include <atomic>

#include "heat1d_device.h"
#include "heat1d_launch.h"
#include "heat1d_rod.h"
#include "heat1d_steps.h"

namespace heat1d {

// ---------------------------------------------------------------------------
// kRing: the periodic ring of Section 5.3 (every point updated, point 0 and
// point N-1 neighbours); otherwise the Dirichlet rod.
template <typename F, bool kRing>
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
    v[0] = i0 > 0 ? src[i0 - 1] : (kRing ? src[N - 1] : F(0));
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
    F o[V];
    if constexpr (kRing) {
      // the point after N-1 is point 0
#pragma unroll
      for (int e = 1; e < V + 2; ++e)
        if (i0 - 1 + e == N) v[e] = src[0];
#pragma unroll
      for (int e = 0; e < V; ++e) o[e] = eq3_step(v[e], v[e + 1], v[e + 2], r);
    } else {
      // the ends hold c1 / cN at every step, including in the initial state
#pragma unroll
      for (int e = 0; e < V + 2; ++e) {
        const int64_t g = i0 - 1 + e;
        v[e] = (g == 0) ? c1 : (g == N - 1) ? cN : v[e];
      }
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const int64_t i = i0 + e;
        o[e] = (i == 0) ? c1 : (i == N - 1) ? cN : eq3_step(v[e], v[e + 1], v[e + 2], r);
      }
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

// One wavefront per tile, one launch per pass.
template <typename F, int M, int S>
__global__ __launch_bounds__(256) void sync_tiled_kernel(const F* __restrict__ in,
                                                         F* __restrict__ out, int64_t N,
                                                         int64_t total_tiles,
                                                         int64_t tiles_per_rod, int H, int steps,
                                                         F r, F c1, F cN, StepWeights<F> sw,
                                                         int aligned) {
  constexpr int L = kWave * M;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wid = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
  if (wid >= total_tiles) return;
  const int64_t rod = wid / tiles_per_rod;
  const int64_t t = wid - rod * tiles_per_rod;
  F u[M];
  load_points<F, M>(u, in + rod * N, t * (L - 2 * H) + lane * M, N, aligned != 0);
  tile_pass<F, M, S>(u, out + rod * N, N, t, tiles_per_rod, H, steps, r, c1, cN, sw,
                            aligned != 0, lane);
}

// Load lane's M points of a ring of n points starting at ring index g0, taken
// modulo n (g0 may be negative or past n; any n >= 1): one 64-bit remainder
// per lane, then an index that wraps from n-1 to 0.
template <typename F, int M>
__device__ __forceinline__ void load_ring_points(F (&u)[M], const F* __restrict__ src, int64_t g0,
                                                 int64_t n) {
  int64_t g = g0 % n;
  if (g < 0) g += n;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    u[j] = src[g];
    g = (g + 1 == n) ? 0 : g + 1;
  }
}

// The periodic ring (Section 5.3) in the tiled geometry: every tile is an
// interior tile.  Tile t writes the ring points [t*Wout, (t+1)*Wout) (cut at N)
// and loads the L points from t*Wout - H on, taken modulo N, so the first and
// last tiles read across the seam between point N-1 and point 0; `steps` <= H
// steps of the periodic extension are exact on the middle L - 2H points.
// Tiles that do not cross the seam load whole vectors.
template <typename F, int M, int S>
__global__ __launch_bounds__(256) void sync_ring_kernel(const F* __restrict__ in,
                                                        F* __restrict__ out, int64_t N,
                                                        int64_t total_tiles, int64_t tiles_per_rod,
                                                        int H, int steps, F r,
                                                        StepWeights<F> sw, int aligned) {
  constexpr int L = kWave * M;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wid = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
  if (wid >= total_tiles) return;
  const int64_t rod = wid / tiles_per_rod;
  const int64_t t = wid - rod * tiles_per_rod;
  const int Wout = L - 2 * H;
  const int64_t base = t * Wout - H;  // ring index of the tile's local point 0
  const F* __restrict__ src = in + rod * N;
  const int q0 = lane * M;
  F u[M];
  if (base >= 0 && base + L <= N)
    load_points<F, M>(u, src, base + q0, N, aligned != 0);
  else
    load_ring_points<F, M>(u, src, base + q0, N);
  advance_interior<F, M, S>(u, steps, r, sw);
  const int64_t hi = N - t * Wout;  // points of the ring left from this tile's first output
  const int ohi = H + (hi < Wout ? (int)hi : Wout);
  // local q holds ring point base + q; the output range [H, ohi) starts at t*Wout
  store_points<F, M>(u, out + rod * N, base + q0, q0, H, ohi,
                     aligned != 0 && base >= 0 && ((base % Vec<F>::n) == 0));
}

// A tile holding neither rod end: `steps` steps, then store [H, L-H).
template <typename F, int M, int S>
__device__ __forceinline__ void interior_pass(F (&u)[M], F* __restrict__ dst, int64_t base, int H,
                                              int steps, F r, const StepWeights<F>& sw,
                                              int lane) {
  constexpr int L = kWave * M;
  advance_interior<F, M, S>(u, steps, r, sw);
  const int q0 = lane * M;
  store_points<F, M>(u, dst, base + q0, q0, H, L - H, true);
}

// A tile holding a rod end, in the pipelined kernel's geometry: the left tile
// starts at point 0 and the right tile ends at point N-1, so both pinned points
// sit at fixed registers (u[0] of lane 0, u[M-1] of lane 63) and cost one
// select per step each.  Stores [lo, hi).
template <typename F, int M>
__device__ __forceinline__ void end_pass(F (&u)[M], F* __restrict__ dst, int64_t gbase, int lo,
                                         int hi, int steps, F r, F c1, F cN, bool right,
                                         int lane) {
  const bool pin_l = !right && lane == 0;
  const bool pin_r = right && lane == kWave - 1;
  u[0] = pin_l ? c1 : u[0];
  u[M - 1] = pin_r ? cN : u[M - 1];
  for (int s = 0; s < steps; ++s) {
    const F left = from_lower_lane(u[M - 1]);
    const F right_v = from_upper_lane(u[0]);
    lane_step<F, M>(u, left, right_v, r);
    u[0] = pin_l ? c1 : u[0];
    u[M - 1] = pin_r ? cN : u[M - 1];
  }
  const int q0 = lane * M;
  store_points<F, M>(u, dst, gbase + q0, q0, lo, hi, true);
}

// Persistent form of the same pass for rods longer than one tile: a grid of at
// most the resident wavefronts, wavefront w taking tiles w, w + W, w + 2W, ...
// of one index space (W = wavefronts in the grid).  Indices [0, 2*nrods) are
// the two end tiles of every rod; the indices after them are the interior
// tiles (tiles 1 .. tiles_per_rod-2 of the tiled geometry).  The right end tile
// is shifted to end exactly at point N-1 and writes what the interior tiles
// leave, [(tiles_per_rod-1)*Wout + H, N).  Interior tiles run as a pipeline:
// each wavefront loads its next tile into a second register set while it
// computes the current one, so HBM transfers overlap the arithmetic instead of
// alternating with it across the whole chip.  The two sets A and B swap roles
// every tile (the loop body is written out twice, so no register copies are
// needed).  The prefetch is issued on every path (past the last tile it reads
// the last interior tile again), which lets the compiler wait for exactly the
// loads a tile needs and never for the prefetch in flight.
template <typename F, int M, int S>
__global__ __launch_bounds__(256) void sync_pipelined_kernel(
    const F* __restrict__ in, F* __restrict__ out, int64_t N, int64_t nrods,
    int64_t tiles_per_rod, int H, int steps, F r, F c1, F cN, StepWeights<F> sw) {
  constexpr int L = kWave * M;
  const int lane = threadIdx.x & (kWave - 1);
  const int Wout = L - 2 * H;
  const int64_t W = (int64_t)gridDim.x * (blockDim.x / kWave);
  const int64_t n_edge = 2 * nrods;
  const int64_t inner_per_rod = tiles_per_rod - 2;
  const int64_t n_inner = inner_per_rod * nrods;
  const int lo_right = (int)((tiles_per_rod - 1) * Wout + H - (N - L));

  int64_t idx = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
  for (; idx < n_edge; idx += W) {
    const int64_t rod = idx >> 1;
    const bool right = (idx & 1) != 0;
    const int64_t gbase = right ? N - L : 0;
    F e[M];
    load_points_vec<F, M>(e, in + rod * N, gbase + lane * M, N);
    end_pass<F, M>(e, out + rod * N, gbase, right ? lo_right : 0, right ? L : L - H, steps, r, c1,
                   cN, right, lane);
  }
  int64_t ia = idx - n_edge;
  if (ia >= n_inner) return;

  // interior tile i of the whole batch: rod i / inner_per_rod, tile 1 + remainder
  auto locate = [&](int64_t i, int64_t& rod, int64_t& g) {
    i = i < n_inner ? i : n_inner - 1;
    rod = i / inner_per_rod;
    g = (1 + i - rod * inner_per_rod) * Wout;
  };
  F a[M], b[M];
  int64_t rod_a, g_a, rod_b, g_b;
  locate(ia, rod_a, g_a);
  load_points_vec<F, M>(a, in + rod_a * N, g_a + lane * M, N);
  for (;;) {
    const int64_t ib = ia + W;
    locate(ib, rod_b, g_b);
    load_points_vec<F, M>(b, in + rod_b * N, g_b + lane * M, N);
    interior_pass<F, M, S>(a, out + rod_a * N, g_a, H, steps, r, sw, lane);
    if (ib >= n_inner) break;
    ia = ib + W;
    locate(ia, rod_a, g_a);
    load_points_vec<F, M>(a, in + rod_a * N, g_a + lane * M, N);
    interior_pass<F, M, S>(b, out + rod_b * N, g_b, H, steps, r, sw, lane);
    if (ia >= n_inner) break;
  }
}

// ---------------------------------------------------------------------------
// Wide tiles: a workgroup of G wavefronts holds one tile of G*64*M points,
// wavefront w the points [w*64M, (w+1)*64M).  Inside a wavefront neighbours
// travel by DPP as in the tiled kernel; the points across a wavefront boundary
// are traded through LDS once per sweep (a double-buffered slot per wavefront
// and side, one barrier per sweep).  The halo is paid once per workgroup
// instead of once per wavefront: at T = 96 and M = 32 a tile of one
// wavefront recomputes 2H/(L-2H) = 10% of its points, a tile of four 2.4%.
template <typename F>
struct WideXch {
  F x[2][8][2][8];  // [parity][wavefront][first, last][up to 8 points]
};

// Neighbours of the lane's points for a sweep of depth D: lo[d] = point -1-d,
// hi[d] = point M+d.  Lanes 0 and 63 take the adjacent wavefront's edge points
// from LDS (zeros at the tile's own edges, inside its halo).
template <typename F, int M, int D, int G>
__device__ __forceinline__ void wide_neighbours(const F (&u)[M], F (&lo)[D], F (&hi)[D],
                                                WideXch<F>& xs, int par, int wave, int lane) {
  if (lane == 0) {
#pragma unroll
    for (int d = 0; d < D; ++d) xs.x[par][wave][0][d] = u[d];
  }
  if (lane == kWave - 1) {
#pragma unroll
    for (int d = 0; d < D; ++d) xs.x[par][wave][1][d] = u[M - D + d];
  }
  __syncthreads();
#pragma unroll
  for (int d = 0; d < D; ++d) {
    lo[d] = from_lower_lane(u[M - 1 - d]);
    hi[d] = from_upper_lane(u[d]);
  }
  if (lane == 0) {
#pragma unroll
    for (int d = 0; d < D; ++d) lo[d] = wave > 0 ? xs.x[par][wave - 1][1][D - 1 - d] : F(0);
  }
  if (lane == kWave - 1) {
#pragma unroll
    for (int d = 0; d < D; ++d) hi[d] = wave + 1 < G ? xs.x[par][wave + 1][0][d] : F(0);
  }
#pragma unroll
  for (int d = 0; d < D; ++d) asm volatile("" : "+v"(lo[d]), "+v"(hi[d]));
}

// `steps` steps of a tile holding no pinned point: pairs of fused S-step sweeps
// (the second sweep reads back into u, so no register copies), then single
// steps.  Every wavefront of the workgroup calls it with the same `steps`.
template <typename F, int M, int S, int G>
__device__ __forceinline__ void wide_interior(F (&u)[M], WideXch<F>& xs, int& par, int steps, F r,
                                              const StepWeights<F>& sw, int wave, int lane) {
  int s = 0;
  if constexpr (S > 1) {
    StepWeights<F> vw = sw;
#pragma unroll
    for (int d = 0; d <= S; ++d) asm volatile("" : "+v"(vw.w[d]));
    F v[M];
    for (; s + 2 * S <= steps; s += 2 * S) {
      F lo[S], hi[S];
      wide_neighbours<F, M, S, G>(u, lo, hi, xs, par, wave, lane);
      par ^= 1;
      lane_multistep_with<F, M, S>(u, v, vw, lo, hi);
      wide_neighbours<F, M, S, G>(v, lo, hi, xs, par, wave, lane);
      par ^= 1;
      lane_multistep_with<F, M, S>(v, u, vw, lo, hi);
    }
  }
  for (; s < steps; ++s) {
    F lo[1], hi[1];
    wide_neighbours<F, M, 1, G>(u, lo, hi, xs, par, wave, lane);
    par ^= 1;
    lane_step<F, M>(u, lo[0], hi[0], r);
  }
}

// Four wavefronts per SIMD (two workgroups of 8 per CU): at most 128 VGPRs,
// which the 8-step sweep at M = 32 needs to be told (it would take 131 and
// fall to three wavefronts per SIMD, i.e. one 8-wavefront workgroup per CU).
template <typename F, int M, int S, int G>
__global__ __launch_bounds__(G * 64) __attribute__((amdgpu_waves_per_eu(4))) void sync_wide_kernel(const F* __restrict__ in,
                                                           F* __restrict__ out, int64_t N,
                                                           int64_t total_tiles,
                                                           int64_t tiles_per_rod, int H,
                                                           int steps, F r, F c1, F cN,
                                                           StepWeights<F> sw, int aligned) {
  constexpr int LW = kWave * M;  // points per wavefront
  constexpr int L = G * LW;      // points per tile
  __shared__ WideXch<F> xs;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int64_t tile = blockIdx.x;
  if (tile >= total_tiles) return;
  const int64_t rod = tile / tiles_per_rod;
  const int64_t t = tile - rod * tiles_per_rod;
  const int Wout = L - 2 * H;
  const int64_t base = t * Wout;
  const int q0 = wave * LW + lane * M;
  F u[M];
  load_points<F, M>(u, in + rod * N, base + q0, N, aligned != 0);
  const bool left_end = (t == 0);
  const int64_t qN64 = N - 1 - base;
  const bool right_end = qN64 < L;
  const int lo_t = left_end ? 0 : H;
  const int hi_t = (t == tiles_per_rod - 1) ? (int)(N - base) : (L - H);
  int par = 0;
  if (left_end || right_end) {
    // single steps, both rod ends re-imposed after every step
    const int qN = right_end ? (int)qN64 : 0;
    const int wN = qN / LW;
    const int lN = (qN / M) % kWave;
    const int jN = uniform(qN % M);
    const bool pin_l = left_end && wave == 0;
    const bool pin_r = right_end && wave == wN;
    if (pin_l) u[0] = (lane == 0) ? c1 : u[0];
    if (pin_r) set_point<F, M>(u, jN, lane == lN, cN);
    for (int s = 0; s < steps; ++s) {
      F lo[1], hi[1];
      wide_neighbours<F, M, 1, G>(u, lo, hi, xs, par, wave, lane);
      par ^= 1;
      lane_step<F, M>(u, lo[0], hi[0], r);
      if (pin_l) u[0] = (lane == 0) ? c1 : u[0];
      if (pin_r) set_point<F, M>(u, jN, lane == lN, cN);
    }
  } else {
    wide_interior<F, M, S, G>(u, xs, par, steps, r, sw, wave, lane);
  }
  store_points<F, M>(u, out + rod * N, base + q0, q0, lo_t, hi_t, aligned != 0);
}

// The periodic ring (Section 5.3) in wide tiles: the ring tiles of
// sync_ring_kernel with G wavefronts per tile.  Tile t writes the ring points
// [t*Wout, (t+1)*Wout) (cut at N) from the L points loaded from t*Wout - H on,
// modulo N; every tile runs the interior sweeps.
template <typename F, int M, int S, int G>
__global__ __launch_bounds__(G * 64) __attribute__((amdgpu_waves_per_eu(4))) void sync_wide_ring_kernel(
    const F* __restrict__ in, F* __restrict__ out, int64_t N, int64_t total_tiles,
    int64_t tiles_per_rod, int H, int steps, F r, StepWeights<F> sw, int aligned) {
  constexpr int LW = kWave * M;
  constexpr int L = G * LW;
  __shared__ WideXch<F> xs;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int64_t tile = blockIdx.x;
  if (tile >= total_tiles) return;
  const int64_t rod = tile / tiles_per_rod;
  const int64_t t = tile - rod * tiles_per_rod;
  const int Wout = L - 2 * H;
  const int64_t base = t * Wout - H;  // ring index of the tile's local point 0
  const F* __restrict__ src = in + rod * N;
  const int q0 = wave * LW + lane * M;
  F u[M];
  if (base >= 0 && base + L <= N)
    load_points<F, M>(u, src, base + q0, N, aligned != 0);
  else
    load_ring_points<F, M>(u, src, base + q0, N);
  int par = 0;
  wide_interior<F, M, S, G>(u, xs, par, steps, r, sw, wave, lane);
  const int64_t hi = N - t * Wout;  // ring points from this tile's first output on
  const int ohi = H + (hi < Wout ? (int)hi : Wout);
  store_points<F, M>(u, out + rod * N, base + q0, q0, H, ohi,
                     aligned != 0 && base >= 0 && ((base % Vec<F>::n) == 0));
}

// ---------------------------------------------------------------------------
template <typename F, int M>
__global__ __launch_bounds__(1024) void sync_resident_kernel(const F* __restrict__ in,
                                                             F* __restrict__ out, int64_t N,
                                                             int K, F r, F c1, F cN,
                                                             int aligned) {
  __shared__ F lds[8 * 16];
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
                            double r, double c1, double cN, hipStream_t s, bool ring) {
  const int V = dtype == 0 ? 4 : 2;
  const int64_t nchunks = (N + V - 1) / V;
  int64_t blocks = (nchunks + 255) / 256;
  if (blocks > 65535) blocks = 65535;
  const int aligned = is_aligned16(in) && is_aligned16(out) && (nrods == 1 || N % V == 0);
  dim3 grid((unsigned)blocks, (unsigned)nrods);
  if (dtype == 0) {
    if (ring)
      hipLaunchKernelGGL((sync_step_kernel<float, true>), grid, dim3(256), 0, s, (const float*)in,
                         (float*)out, N, (float)r, (float)c1, (float)cN, aligned);
    else
      hipLaunchKernelGGL((sync_step_kernel<float, false>), grid, dim3(256), 0, s,
                         (const float*)in, (float*)out, N, (float)r, (float)c1, (float)cN,
                         aligned);
  } else {
    if (ring)
      hipLaunchKernelGGL((sync_step_kernel<double, true>), grid, dim3(256), 0, s,
                         (const double*)in, (double*)out, N, r, c1, cN, aligned);
    else
      hipLaunchKernelGGL((sync_step_kernel<double, false>), grid, dim3(256), 0, s,
                         (const double*)in, (double*)out, N, r, c1, cN, aligned);
  }
  return hipGetLastError();
}

TileGeom ring_geometry(int dtype, int M, int T, int64_t N) {
  TileGeom g = tile_geometry(dtype, M, T, N);
  if (g.Wout > 0) g.tiles_per_rod = (N + g.Wout - 1) / g.Wout;
  return g;
}

template <typename F, int M, int S>
static void ring_launch(const TileGeom& g, const void* in, void* out, int64_t N, int64_t nrods,
                        int steps, double r, hipStream_t s) {
  const int64_t total = g.tiles_per_rod * nrods;
  const int wpb = 4;
  const int64_t blocks = (total + wpb - 1) / wpb;
  const int V = Vec<F>::n;
  const int aligned = is_aligned16(in) && is_aligned16(out) && (nrods == 1 || N % V == 0);
  hipLaunchKernelGGL((sync_ring_kernel<F, M, S>), dim3((unsigned)blocks), dim3(wpb * kWave), 0, s,
                     (const F*)in, (F*)out, N, total, g.tiles_per_rod, g.H, steps, (F)r,
                     step_weights<F>(r, S), aligned);
}

hipError_t launch_sync_ring(int dtype, const TileGeom& g, const void* in, void* out, int64_t N,
                            int64_t nrods, int steps, double r, int fuse, hipStream_t s) {
  if (steps > g.H || g.tiles_per_rod <= 0 || g.Wout <= 0 || !fused_supports(dtype, g.M, fuse) ||
      g.tiles_per_rod * nrods > 0x7fffffffLL)
    return hipErrorInvalidValue;
#define HEAT1D_RING(FT, MM, SS)                                       \
  case (MM) * 8 + (SS):                                               \
    ring_launch<FT, MM, SS>(g, in, out, N, nrods, steps, r, s);       \
    break;
  if (dtype == 0) {
    switch (g.M * 8 + fuse) {
      HEAT1D_FOR_EACH_F32(HEAT1D_RING)
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (g.M * 8 + fuse) {
      HEAT1D_FOR_EACH_F64(HEAT1D_RING)
      default: return hipErrorInvalidValue;
    }
  }
#undef HEAT1D_RING
  return hipGetLastError();
}

bool fused_supports(int dtype, int M, int S) {
  if (S == 1) return tiled_supports(dtype, M);
  if (S != 2 && S != 4) return false;
  if (dtype == 0) return M == 16 || M == 32 || M == 48 || M == 64;
  return M == 8 || M == 16 || M == 24 || M == 32;
}

template <typename F, int M, int S>
static void tiled_launch(const TileGeom& g, const void* in, void* out, int64_t N, int64_t nrods,
                         int steps, double r, double c1, double cN, hipStream_t s) {
  const int64_t total = g.tiles_per_rod * nrods;
  const int wpb = 4;
  const int64_t blocks = (total + wpb - 1) / wpb;
  const int V = Vec<F>::n;
  const int aligned = is_aligned16(in) && is_aligned16(out) && (nrods == 1 || N % V == 0);
  hipLaunchKernelGGL((sync_tiled_kernel<F, M, S>), dim3((unsigned)blocks), dim3(wpb * kWave), 0,
                     s, (const F*)in, (F*)out, N, total, g.tiles_per_rod, g.H, steps, (F)r,
                     (F)c1, (F)cN, step_weights<F>(r, S), aligned);
}

hipError_t launch_sync_tiled(int dtype, const TileGeom& g, const void* in, void* out, int64_t N,
                             int64_t nrods, int steps, double r, double c1, double cN, int fuse,
                             hipStream_t s) {
  if (steps > g.H || g.tiles_per_rod <= 0 || !fused_supports(dtype, g.M, fuse))
    return hipErrorInvalidValue;
#define HEAT1D_TILED(FT, MM, SS)                                               \
  case (MM) * 8 + (SS):                                                        \
    tiled_launch<FT, MM, SS>(g, in, out, N, nrods, steps, r, c1, cN, s);      \
    break;
  if (dtype == 0) {
    switch (g.M * 8 + fuse) {
      HEAT1D_FOR_EACH_F32(HEAT1D_TILED)
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (g.M * 8 + fuse) {
      HEAT1D_FOR_EACH_F64(HEAT1D_TILED)
      default: return hipErrorInvalidValue;
    }
  }
#undef HEAT1D_TILED
  return hipGetLastError();
}

// Wide tiles: G = 4 or 8 wavefronts per tile, (M, S) pairs below.
bool wide_supports(int dtype, int M, int S, int G) {
  if (S == 8) return dtype == 0 && (M == 16 || M == 32) && (G == 4 || G == 8);
  if ((G != 4 && G != 8) || (S != 1 && S != 4)) return false;
  if (dtype == 0) return M == 16 || M == 32 || (M == 48 && G == 4);
  return M == 8 || M == 16 || (M == 24 && G == 4);
}

template <typename F, int M, int S, int G>
static void wide_launch(const TileGeom& g, const void* in, void* out, int64_t N, int64_t nrods,
                        int steps, double r, double c1, double cN, hipStream_t s) {
  const int64_t total = g.tiles_per_rod * nrods;
  const int V = Vec<F>::n;
  const int aligned = is_aligned16(in) && is_aligned16(out) && (nrods == 1 || N % V == 0);
  hipLaunchKernelGGL((sync_wide_kernel<F, M, S, G>), dim3((unsigned)total), dim3(G * kWave), 0,
                     s, (const F*)in, (F*)out, N, total, g.tiles_per_rod, g.H, steps, (F)r,
                     (F)c1, (F)cN, step_weights<F>(r, S), aligned);
}

hipError_t launch_sync_wide(int dtype, const TileGeom& g, int M, int G, const void* in, void* out,
                            int64_t N, int64_t nrods, int steps, double r, double c1, double cN,
                            int fuse, hipStream_t s) {
  if (steps > g.H || g.tiles_per_rod <= 0 || !wide_supports(dtype, M, fuse, G) ||
      g.M != M * G || g.tiles_per_rod * nrods > 0x7fffffffLL)
    return hipErrorInvalidValue;
#define HEAT1D_WIDE(FT, MM, SS, GG)                                                   \
  case ((MM) * 8 + (SS)) * 16 + (GG):                                                 \
    wide_launch<FT, MM, SS, GG>(g, in, out, N, nrods, steps, r, c1, cN, s);          \
    break;
  const int key = (M * 8 + fuse) * 16 + G;
  if (dtype == 0) {
    switch (key) {
      HEAT1D_WIDE(float, 16, 1, 4) HEAT1D_WIDE(float, 32, 1, 4) HEAT1D_WIDE(float, 48, 1, 4)
      HEAT1D_WIDE(float, 16, 4, 4) HEAT1D_WIDE(float, 32, 4, 4) HEAT1D_WIDE(float, 48, 4, 4)
      HEAT1D_WIDE(float, 16, 1, 8) HEAT1D_WIDE(float, 32, 1, 8)
      HEAT1D_WIDE(float, 16, 4, 8) HEAT1D_WIDE(float, 32, 4, 8)
      HEAT1D_WIDE(float, 16, 8, 4) HEAT1D_WIDE(float, 32, 8, 4)
      HEAT1D_WIDE(float, 16, 8, 8) HEAT1D_WIDE(float, 32, 8, 8)
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (key) {
      HEAT1D_WIDE(double, 8, 1, 4) HEAT1D_WIDE(double, 16, 1, 4) HEAT1D_WIDE(double, 24, 1, 4)
      HEAT1D_WIDE(double, 8, 4, 4) HEAT1D_WIDE(double, 16, 4, 4) HEAT1D_WIDE(double, 24, 4, 4)
      HEAT1D_WIDE(double, 8, 1, 8) HEAT1D_WIDE(double, 16, 1, 8)
      HEAT1D_WIDE(double, 8, 4, 8) HEAT1D_WIDE(double, 16, 4, 8)
      default: return hipErrorInvalidValue;
    }
  }
#undef HEAT1D_WIDE
  return hipGetLastError();
}

template <typename F, int M, int S, int G>
static void wide_ring_launch(const TileGeom& g, const void* in, void* out, int64_t N,
                             int64_t nrods, int steps, double r, hipStream_t s) {
  const int64_t total = g.tiles_per_rod * nrods;
  const int V = Vec<F>::n;
  const int aligned = is_aligned16(in) && is_aligned16(out) && (nrods == 1 || N % V == 0);
  hipLaunchKernelGGL((sync_wide_ring_kernel<F, M, S, G>), dim3((unsigned)total), dim3(G * kWave),
                     0, s, (const F*)in, (F*)out, N, total, g.tiles_per_rod, g.H, steps, (F)r,
                     step_weights<F>(r, S), aligned);
}

hipError_t launch_sync_wide_ring(int dtype, const TileGeom& g, int M, int G, const void* in,
                                 void* out, int64_t N, int64_t nrods, int steps, double r,
                                 int fuse, hipStream_t s) {
  if (steps > g.H || g.tiles_per_rod <= 0 || g.Wout <= 0 || !wide_supports(dtype, M, fuse, G) ||
      g.M != M * G || g.tiles_per_rod * nrods > 0x7fffffffLL)
    return hipErrorInvalidValue;
#define HEAT1D_WIDE_RING(FT, MM, SS, GG)                                   \
  case ((MM) * 8 + (SS)) * 16 + (GG):                                      \
    wide_ring_launch<FT, MM, SS, GG>(g, in, out, N, nrods, steps, r, s);   \
    break;
  const int key = (M * 8 + fuse) * 16 + G;
  if (dtype == 0) {
    switch (key) {
      HEAT1D_WIDE_RING(float, 16, 1, 4) HEAT1D_WIDE_RING(float, 32, 1, 4)
      HEAT1D_WIDE_RING(float, 48, 1, 4) HEAT1D_WIDE_RING(float, 16, 4, 4)
      HEAT1D_WIDE_RING(float, 32, 4, 4) HEAT1D_WIDE_RING(float, 48, 4, 4)
      HEAT1D_WIDE_RING(float, 16, 1, 8) HEAT1D_WIDE_RING(float, 32, 1, 8)
      HEAT1D_WIDE_RING(float, 16, 4, 8) HEAT1D_WIDE_RING(float, 32, 4, 8)
      HEAT1D_WIDE_RING(float, 16, 8, 4) HEAT1D_WIDE_RING(float, 32, 8, 4)
      HEAT1D_WIDE_RING(float, 16, 8, 8) HEAT1D_WIDE_RING(float, 32, 8, 8)
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (key) {
      HEAT1D_WIDE_RING(double, 8, 1, 4) HEAT1D_WIDE_RING(double, 16, 1, 4)
      HEAT1D_WIDE_RING(double, 24, 1, 4) HEAT1D_WIDE_RING(double, 8, 4, 4)
      HEAT1D_WIDE_RING(double, 16, 4, 4) HEAT1D_WIDE_RING(double, 24, 4, 4)
      HEAT1D_WIDE_RING(double, 8, 1, 8) HEAT1D_WIDE_RING(double, 16, 1, 8)
      HEAT1D_WIDE_RING(double, 8, 4, 8) HEAT1D_WIDE_RING(double, 16, 4, 8)
      default: return hipErrorInvalidValue;
    }
  }
#undef HEAT1D_WIDE_RING
  return hipGetLastError();
}

// The pipelined pass moves whole 16-byte vectors only and needs rods longer
// than one tile.
bool pipelined_applies(int dtype, const TileGeom& g, const void* in, const void* out, int64_t N) {
  const int V = dtype == 0 ? 4 : 2;
  return is_aligned16(in) && is_aligned16(out) && N % V == 0 && g.tiles_per_rod >= 2 &&
         N > g.L;
}

// Resident 256-thread workgroups per CU of the pipelined kernel, queried once
// per instantiation.
template <typename F, int M, int S>
static int pipelined_blocks_per_cu() {
  static std::atomic<int> cached{0};
  int nb = cached.load(std::memory_order_relaxed);
  if (nb > 0) return nb;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sync_pipelined_kernel<F, M, S>, 256, 0) !=
          hipSuccess ||
      nb < 1)
    nb = 1;
  cached.store(nb, std::memory_order_relaxed);
  return nb;
}

template <typename F, int M, int S>
static hipError_t pipelined_launch(const TileGeom& g, const void* in, void* out, int64_t N,
                                   int64_t nrods, int steps, double r, double c1, double cN,
                                   hipStream_t s) {
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int wpb = 4;
  const int64_t resident =
      (int64_t)pipelined_blocks_per_cu<F, M, S>() * (ncu > 0 ? ncu : 1) * wpb;
  // every resident slot filled: the dispatcher deals workgroups round-robin
  // over the CUs, so the wavefronts that get one tile more than the others are
  // spread evenly over the SIMDs (trimming the grid would leave some CUs with
  // fewer wavefronts and the rest with a longer queue)
  const int64_t n_all = g.tiles_per_rod * nrods;
  const int64_t waves = std::min<int64_t>(resident, n_all);
  const int64_t blocks = (waves + wpb - 1) / wpb;
  hipLaunchKernelGGL((sync_pipelined_kernel<F, M, S>), dim3((unsigned)blocks),
                     dim3(wpb * kWave), 0, s, (const F*)in, (F*)out, N, nrods, g.tiles_per_rod,
                     g.H, steps, (F)r, (F)c1, (F)cN, step_weights<F>(r, S));
  return hipGetLastError();
}

hipError_t launch_sync_pipelined(int dtype, const TileGeom& g, const void* in, void* out,
                                 int64_t N, int64_t nrods, int steps, double r, double c1,
                                 double cN, int fuse, hipStream_t s) {
  if (steps > g.H || g.tiles_per_rod <= 0 || !fused_supports(dtype, g.M, fuse))
    return hipErrorInvalidValue;
  if (!pipelined_applies(dtype, g, in, out, N)) return hipErrorInvalidValue;
#define HEAT1D_PIPE(FT, MM, SS)                                                  \
  case (MM) * 8 + (SS):                                                          \
    return pipelined_launch<FT, MM, SS>(g, in, out, N, nrods, steps, r, c1, cN, s);
  if (dtype == 0) {
    switch (g.M * 8 + fuse) {
      HEAT1D_FOR_EACH_F32(HEAT1D_PIPE)
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (g.M * 8 + fuse) {
      HEAT1D_FOR_EACH_F64(HEAT1D_PIPE)
      default: return hipErrorInvalidValue;
    }
  }
#undef HEAT1D_PIPE
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
