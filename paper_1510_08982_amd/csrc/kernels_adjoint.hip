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
//    the starts of its sub-stretches of S2 steps are recomputed into a small
//    HBM buffer (tiled passes of depth S2);
//  * stretch_kernel handles one sub-stretch per launch: for each tile it loads
//    the sub-stretch's first state, recomputes the S2 steps that follow and
//    keeps, in registers, the discrete Laplacian of each of those states (S2 x
//    M values per lane, no HBM traffic), then walks the S2 steps backwards
//    with lambda in registers, adding lambda(k+1) times the Laplacian of u(k).
// The Laplacian a + b - 2c is the inner term of the forward step itself
// (u(k+1) = c + r(a + b - 2c)), so keeping it costs no arithmetic, and the
// backward step needs one fused multiply-add per point for dL/dr.
//
// The kernel is persistent: each wavefront takes tiles w, w+W, w+2W, ... and
// loads the next tile's two input states before it computes the current one,
// so the load latency is hidden behind a tile of arithmetic.  HBM traffic is
// about three states per sub-stretch in the kernel plus two per sub-stretch
// start recomputed, instead of two per step.  Each tile sums the dL/dr terms
// of the points it owns only (no double counting across overlapping halos)
// into one double per tile; the partial sums are reduced in a fixed order, so
// dL/dr is deterministic.
#include "heat1d_device.h"
#include "heat1d_launch.h"

#include <atomic>

namespace heat1d {

// Steps per register-resident sub-stretch and points per lane.  The
// Laplacians take KS x M registers per lane: 192 (FP32) and 128 (FP64), which
// with the two input states of the next tile still leaves two wavefronts per
// SIMD.
template <typename F> struct StretchShape;
template <> struct StretchShape<float> { static constexpr int M = 8, KS = 24; };
template <> struct StretchShape<double> { static constexpr int M = 4, KS = 16; };

// Lane neighbours for the sub-stretch steps.  FP32 goes through the LDS
// crossbar (ds_bpermute, no LDS storage): with only 8 points per lane the
// exchange sits on every step's critical path, and there it measured a few
// percent faster than the DPP wavefront shift.  Lane 0 receives lane 63's
// value and lane 63 lane 0's: both are tile edges, whose values the halo
// absorbs (or pinned rod ends).  FP64 keeps the DPP shift.
__device__ __forceinline__ float nb_lower(float x) {
  const int l = (int)(threadIdx.x & (kWave - 1));
  return __int_as_float(__builtin_amdgcn_ds_bpermute(((l + kWave - 1) & (kWave - 1)) << 2,
                                                     __float_as_int(x)));
}
__device__ __forceinline__ float nb_upper(float x) {
  const int l = (int)(threadIdx.x & (kWave - 1));
  return __int_as_float(
      __builtin_amdgcn_ds_bpermute(((l + 1) & (kWave - 1)) << 2, __float_as_int(x)));
}
__device__ __forceinline__ double nb_lower(double x) { return from_lower_lane(x); }
__device__ __forceinline__ double nb_upper(double x) { return from_upper_lane(x); }

// Deterministic wavefront sum (fixed butterfly order).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

template <typename F>
struct StretchDev {
  const F* u_start;
  const F* lam_in;
  F* lam_out;
  double* partials;     // partials[rod * part_stride + part_off + tile]
  int64_t N;
  int64_t total_tiles;
  int64_t tiles_per_rod;
  int64_t part_stride;
  int64_t part_off;
  int64_t part_rods;    // rods holding partials (the buffer's extent)
  int H;
  int len;
  F r, c1, cN;
  int aligned;
};

// Tile t of a rod covers [t*Wout, t*Wout + L), the geometry of the tiled
// forward kernel, with the halo H >= KS + 1: the Laplacian of u(k0+s) is exact
// on [s+1, L-s-1) of an inner tile and lambda(k0+s) on [len-s, L-len+s), so
// both stay exact on the owned points [H, L-H) for the whole sub-stretch.
// kPipe (aligned buffers, N a multiple of the vector width and at least L, all
// tile and byte counts within 31 bits): the last tile of a rod is moved left to
// end exactly at point N-1 and owns the points from where tile T-2 stops, so
// the pinned point N-1 sits in a fixed register (u[M-1] of lane 63), as point
// 0 does in the first tile (u[0] of lane 0).  Only the last tile ever holds
// point N-1: tile T-2 ends before it.
struct StretchTile {
  int64_t rod;
  int64_t t;
  int64_t base;  // rod index of the tile's first point
  int olo;       // first local point the tile stores
  bool left_end, right_end;
};

template <typename F, int M, bool kPipe>
__device__ __forceinline__ StretchTile stretch_tile_at(const StretchDev<F>& a, int64_t wid) {
  constexpr int L = kWave * M;
  StretchTile g;
  if constexpr (kPipe) {
    const uint32_t w = (uint32_t)wid, tpr = (uint32_t)a.tiles_per_rod;
    g.rod = w / tpr;
    g.t = w - (uint32_t)g.rod * tpr;
  } else {
    g.rod = wid / a.tiles_per_rod;
    g.t = wid - g.rod * a.tiles_per_rod;
  }
  g.left_end = g.t == 0;
  g.right_end = g.t == a.tiles_per_rod - 1;
  const int64_t Wout = L - 2 * a.H;
  g.base = g.t * Wout;
  g.olo = g.left_end ? 0 : a.H;
  if (kPipe && g.right_end && !g.left_end) {
    g.base = a.N - L;
    g.olo = (int)(g.t * Wout + a.H - g.base);
  }
  return g;
}

// Both input states of tile wid.  Unpipelined: points outside [0, N) read as
// 0.  Pipelined: a fixed set of 16-byte loads, all inside the rod, so that a
// prefetch into these registers needs no wait until they are used.
template <typename F, int M, bool kPipe>
__device__ __forceinline__ void stretch_load(const StretchDev<F>& a, int64_t wid, F (&u)[M],
                                             F (&lam)[M], int lane) {
  const StretchTile g = stretch_tile_at<F, M, kPipe>(a, wid);
  const int64_t g0 = g.base + lane * M;
  if constexpr (kPipe) {
    load_points_vec<F, M>(u, a.u_start + g.rod * a.N, g0, a.N);
    load_points_vec<F, M>(lam, a.lam_in + g.rod * a.N, g0, a.N);
  } else {
    load_points<F, M>(u, a.u_start + g.rod * a.N, g0, a.N, a.aligned != 0);
    load_points<F, M>(lam, a.lam_in + g.rod * a.N, g0, a.N, a.aligned != 0);
  }
}

// Buffer resource over `bytes` bytes from `base` (the gfx9 raw-buffer word):
// a store whose offset lies past the end is dropped by the hardware.  Lanes
// that must not store point their offset there, so every lane issues the same
// store instructions and the tile's store count never depends on the lane or
// the tile.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           0x00020000);
}
constexpr uint32_t kDropOffset = 0x80000000u;

using U32x4 = __attribute__((ext_vector_type(4))) uint32_t;
using U32x2 = __attribute__((ext_vector_type(2))) uint32_t;

// Store the 16-byte vectors of the lane's points whose local index lies in
// [lo, hi) (lo, hi and q0 multiples of the vector width, so each vector is
// wholly in or out).
template <typename F, int M>
__device__ __forceinline__ void store_vec_masked(const F (&u)[M], F* rod_base, int64_t N,
                                                 int64_t g0, int q0, int lo, int hi) {
  constexpr int V = Vec<F>::n;
  const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(rod_base, (uint32_t)(N * (int64_t)sizeof(F)));
#pragma unroll
  for (int c = 0; c < M / V; ++c) {
    const int q = q0 + c * V;
    const uint32_t off =
        (q >= lo && q < hi) ? (uint32_t)((g0 + c * V) * (int64_t)sizeof(F)) : kDropOffset;
    U32x4 w;
    __builtin_memcpy(&w, &u[c * V], 16);
    __builtin_amdgcn_raw_buffer_store_b128(w, rs, off, 0, 0);
  }
}

// Re-impose the fixed ends on a lane's points: point 0 (first tile) and point
// N-1 (last tile; at register M-1 of lane 63 when kPipe, else at register jN
// of lane lN).
template <typename F, int M, bool kPipe>
__device__ __forceinline__ void pin_ends(F (&u)[M], bool left_end, bool right_end, int lN, int jN,
                                         int lane, F v_left, F v_right) {
  if (left_end) u[0] = (lane == 0) ? v_left : u[0];
  if (right_end) {
    if constexpr (kPipe)
      u[M - 1] = (lane == kWave - 1) ? v_right : u[M - 1];
    else
      set_point<F, M>(u, jN, lane == lN, v_right);
  }
}

// The sub-stretch of one tile; kEnds: the tile holds a rod end, which is
// re-imposed after every step (c1 / cN on u, zero on lambda).  Tiles away from
// the ends take the kEnds = false copy, which carries none of that code.
// kFull: len == KS, so no step is skipped and the unrolled steps need no test.
//
// Each step first updates the lane's two end points, whose new values its
// neighbour lanes need for the next step, hands them over, and only then
// updates the lane's inner points: the exchange is in flight while the rest of
// the step issues, instead of every step opening with a wait for it.  The
// inner points use the old end values, so every value equals that of the
// plain order (all Laplacians from u(k), then the update) bit for bit.  With
// kPipe the pinned points are end registers (point 0 at u[0] of lane 0, point
// N-1 at u[M-1] of lane 63) and are pinned before the hand-over; the general
// form, whose point N-1 may sit in any register, keeps the plain order.
template <typename F, int M, int KS, bool kEnds, bool kFull, bool kPipe>
__device__ __forceinline__ void stretch_body(const StretchDev<F>& a, F (&u)[M], F (&lam)[M],
                                             F (&acc)[M], bool left_end, bool right_end, int lN,
                                             int jN, int lane) {
  static_assert(M >= 2, "a lane holds at least two points");
  // r in a vector register: a VALU instruction with a scalar operand issues at
  // half rate when such instructions come back to back
  F r = a.r;
  asm volatile("" : "+v"(r));
  // forward: Laplacians of u(k0+s), s < len
  F lap[KS][M];
  if constexpr (kEnds) pin_ends<F, M, kPipe>(u, left_end, right_end, lN, jN, lane, a.c1, a.cN);
  if constexpr (kPipe) {
    static_assert(M >= 4, "the end pairs of a lane do not overlap");
    F left = nb_lower(u[M - 1]);
    F right = nb_upper(u[0]);
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      if (kFull || s < a.len) {
        // the Laplacians of the two end pairs (they read the old end values)
        lap[s][0] = fma_of(F(-2), u[0], left + u[1]);
        lap[s][1] = fma_of(F(-2), u[1], u[0] + u[2]);
        lap[s][M - 2] = fma_of(F(-2), u[M - 2], u[M - 3] + u[M - 1]);
        lap[s][M - 1] = fma_of(F(-2), u[M - 1], u[M - 2] + right);
        if (s + 1 < KS) {
          // u(k0+s+1) = u + r * Laplacian: the forward step, bit for bit
          u[0] = fma_of(r, lap[s][0], u[0]);
          u[M - 1] = fma_of(r, lap[s][M - 1], u[M - 1]);
          if constexpr (kEnds) {
            if (left_end) u[0] = (lane == 0) ? a.c1 : u[0];
            if (right_end) u[M - 1] = (lane == kWave - 1) ? a.cN : u[M - 1];
          }
          left = nb_lower(u[M - 1]);
          right = nb_upper(u[0]);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 2; j < M - 2; ++j) lap[s][j] = fma_of(F(-2), u[j], u[j - 1] + u[j + 1]);
        if (s + 1 < KS) {
#pragma unroll
          for (int j = 1; j < M - 1; ++j) u[j] = fma_of(r, lap[s][j], u[j]);
        }
      }
      // one step at a time: scheduled across steps, the unrolled code keeps
      // far more values live than the registers hold
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      if (kFull || s < a.len) {
        const F left = nb_lower(u[M - 1]);
        const F right = nb_upper(u[0]);
#pragma unroll
        for (int j = 0; j < M; ++j) {
          const F lj = (j == 0) ? left : u[j - 1];
          const F rj = (j + 1 < M) ? u[j + 1] : right;
          lap[s][j] = fma_of(F(-2), u[j], lj + rj);
        }
        if (s + 1 < KS) {
#pragma unroll
          for (int j = 0; j < M; ++j) u[j] = fma_of(r, lap[s][j], u[j]);
          if constexpr (kEnds)
            pin_ends<F, M, kPipe>(u, left_end, right_end, lN, jN, lane, a.c1, a.cN);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }

  // backward: lambda(k0 + len) -> lambda(k0)
  if constexpr (kEnds) pin_ends<F, M, kPipe>(lam, left_end, right_end, lN, jN, lane, F(0), F(0));
#pragma unroll
  for (int j = 0; j < M; ++j) acc[j] = F(0);
  if constexpr (kPipe) {
    F left = nb_lower(lam[M - 1]);
    F right = nb_upper(lam[0]);
#pragma unroll
    for (int s = KS - 1; s >= 0; --s) {
      if (kFull || s < a.len) {
        // lambda(k0+s) = A^T lambda(k0+s+1) (the arithmetic of eq3_step:
        // Laplacian, then the update), the lane's end points first; the
        // dL/dr terms lambda(k0+s+1) * Laplacian of the end points are taken
        // before their lambda is overwritten
        const F d0 = fma_of(F(-2), lam[0], left + lam[1]);
        const F d1 = fma_of(F(-2), lam[1], lam[0] + lam[2]);
        const F d2 = fma_of(F(-2), lam[M - 2], lam[M - 3] + lam[M - 1]);
        const F d3 = fma_of(F(-2), lam[M - 1], lam[M - 2] + right);
        acc[0] = fma_of(lam[0], lap[s][0], acc[0]);
        acc[M - 1] = fma_of(lam[M - 1], lap[s][M - 1], acc[M - 1]);
        lam[0] = fma_of(r, d0, lam[0]);
        lam[M - 1] = fma_of(r, d3, lam[M - 1]);
        if constexpr (kEnds) {
          if (left_end) lam[0] = (lane == 0) ? F(0) : lam[0];
          if (right_end) lam[M - 1] = (lane == kWave - 1) ? F(0) : lam[M - 1];
        }
        if (s > 0) {
          left = nb_lower(lam[M - 1]);
          right = nb_upper(lam[0]);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 1; j < M - 1; ++j) acc[j] = fma_of(lam[j], lap[s][j], acc[j]);
        F d[M];
        d[1] = d1;
        d[M - 2] = d2;
#pragma unroll
        for (int j = 2; j < M - 2; ++j) d[j] = fma_of(F(-2), lam[j], lam[j - 1] + lam[j + 1]);
#pragma unroll
        for (int j = 1; j < M - 1; ++j) lam[j] = fma_of(r, d[j], lam[j]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {
#pragma unroll
    for (int s = KS - 1; s >= 0; --s) {
      if (kFull || s < a.len) {
        // dL/dr term of step k0+s at each point: lambda(k0+s+1) * Laplacian
#pragma unroll
        for (int j = 0; j < M; ++j) acc[j] = fma_of(lam[j], lap[s][j], acc[j]);
        // lambda(k0+s) = A^T lambda(k0+s+1): the same stencil, all Laplacians
        // first, then the update in place (the arithmetic of eq3_step)
        const F left = nb_lower(lam[M - 1]);
        const F right = nb_upper(lam[0]);
        F d[M];
#pragma unroll
        for (int j = 0; j < M; ++j) {
          const F lj = (j == 0) ? left : lam[j - 1];
          const F rj = (j + 1 < M) ? lam[j + 1] : right;
          d[j] = fma_of(F(-2), lam[j], lj + rj);
        }
#pragma unroll
        for (int j = 0; j < M; ++j) lam[j] = fma_of(r, d[j], lam[j]);
        if constexpr (kEnds)
          pin_ends<F, M, kPipe>(lam, left_end, right_end, lN, jN, lane, F(0), F(0));
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

template <typename F, int M, int KS, bool kFull, bool kPipe>
__device__ __forceinline__ void stretch_tile(const StretchDev<F>& a, int64_t wid, F (&u)[M],
                                             F (&lam)[M], int lane) {
  constexpr int L = kWave * M;
  const StretchTile g = stretch_tile_at<F, M, kPipe>(a, wid);
  const int q0 = lane * M;
  F acc[M];
  if (g.left_end || g.right_end) {
    const int qN = g.right_end ? (int)(a.N - 1 - g.base) : 0;
    stretch_body<F, M, KS, true, kFull, kPipe>(a, u, lam, acc, g.left_end, g.right_end, qN / M,
                                               uniform(qN % M), lane);
  } else {
    stretch_body<F, M, KS, false, kFull, kPipe>(a, u, lam, acc, false, false, 0, 0, lane);
  }
  const int ohi = g.right_end ? (int)(a.N - g.base) : (L - a.H);
  if constexpr (kPipe)
    store_vec_masked<F, M>(lam, a.lam_out + g.rod * a.N, a.N, g.base + q0, q0, g.olo, ohi);
  else
    store_points<F, M>(lam, a.lam_out + g.rod * a.N, g.base + q0, q0, g.olo, ohi,
                       a.aligned != 0);

  // points whose dL/dr terms this tile owns: its output range, interior only
  const int lo = g.left_end ? 1 : g.olo;
  const int hi = g.right_end ? (int)(a.N - 1 - g.base) : (L - a.H);
  double part = 0.0;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const int q = q0 + j;
    part += (q >= lo && q < hi) ? (double)acc[j] : 0.0;
  }
  const double tot = wave_sum(part);
  const int64_t pi = g.rod * a.part_stride + a.part_off + g.t;
  if constexpr (kPipe) {
    // lane 0 writes the tile's sum; the other lanes' stores are dropped
    const __amdgpu_buffer_rsrc_t rs =
        buffer_rsrc(a.partials, (uint32_t)(a.part_stride * a.part_rods * 8));
    U32x2 w;
    __builtin_memcpy(&w, &tot, 8);
    __builtin_amdgcn_raw_buffer_store_b64(w, rs, lane == 0 ? (uint32_t)(pi * 8) : kDropOffset,
                                          0, 0);
  } else {
    if (lane == 0) a.partials[pi] = tot;
  }
}

// Each wavefront of the pipelined form alternates two register sets, loading
// the next tile into one while it computes the tile held in the other.
template <typename F, int M, int KS, bool kPipe, bool kFull>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void stretch_kernel(const StretchDev<F> a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t W = (int64_t)gridDim.x * (blockDim.x / kWave);
  // the tile index is wavefront-uniform: kept in scalar registers, the tile
  // loop stays a scalar loop and the geometry scalar arithmetic
  int64_t wid = (int64_t)blockIdx.x * (blockDim.x / kWave) + uniform((int)threadIdx.x / kWave);
  if (wid >= a.total_tiles) return;
  if constexpr (!kPipe) {
    for (; wid < a.total_tiles; wid += W) {
      F u[M], lam[M];
      stretch_load<F, M, false>(a, wid, u, lam, lane);
      stretch_tile<F, M, KS, kFull, false>(a, wid, u, lam, lane);
    }
  } else {
    const int64_t last = a.total_tiles - 1;
    F ua[M], la[M], ub[M], lb[M];
    stretch_load<F, M, true>(a, wid, ua, la, lane);
    for (;;) {
      // the next tile (this one again past the end: the loads stay
      // unconditional)
      stretch_load<F, M, true>(a, wid + W <= last ? wid + W : wid, ub, lb, lane);
      stretch_tile<F, M, KS, kFull, true>(a, wid, ua, la, lane);
      wid += W;
      if (wid > last) break;
      stretch_load<F, M, true>(a, wid + W <= last ? wid + W : wid, ua, la, lane);
      stretch_tile<F, M, KS, kFull, true>(a, wid, ub, lb, lane);
      wid += W;
      if (wid > last) break;
    }
  }
}

// Sums of chunks of the per-tile dL/dr partials.  Block (c, b) adds the
// entries i = c*chunk .. min(n, (c+1)*chunk) - 1 of rod b, in[b*in_stride +
// i*elem_stride]: thread t takes i = c*chunk + t, t + 256, ... in order, then a
// fixed LDS tree combines the 256 sums, so the order never changes between
// runs or devices.  The result goes to out[b*out_stride + c*out_elem_stride].
__global__ __launch_bounds__(256) void reduce_chunks_kernel(const double* in, int64_t n,
                                                            int64_t in_stride, int64_t elem_stride,
                                                            int64_t chunk, double* out,
                                                            int64_t out_stride,
                                                            int64_t out_elem_stride) {
  __shared__ double sh[256];
  const int64_t c = blockIdx.x, b = blockIdx.y;
  const int64_t i0 = c * chunk;
  const int64_t i1 = i0 + chunk < n ? i0 + chunk : n;
  double acc = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) acc += in[b * in_stride + i * elem_stride];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[b * out_stride + c * out_elem_stride] = sh[0];
}

// ---------------------------------------------------------------------------
static bool is_aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

int stretch_steps(int dtype) {
  return dtype == 0 ? StretchShape<float>::KS : StretchShape<double>::KS;
}

static int stretch_pts_per_lane(int dtype) {
  return dtype == 0 ? StretchShape<float>::M : StretchShape<double>::M;
}

TileGeom stretch_geometry(int dtype, int64_t N) {
  return tile_geometry(dtype, stretch_pts_per_lane(dtype), stretch_steps(dtype) + 1, N);
}

template <typename F, bool kPipe, bool kFull>
static int stretch_blocks_per_cu() {
  constexpr int M = StretchShape<F>::M, KS = StretchShape<F>::KS;
  static std::atomic<int> cached{0};
  int nb = cached.load(std::memory_order_relaxed);
  if (nb > 0) return nb;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, stretch_kernel<F, M, KS, kPipe, kFull>, 256, 0) != hipSuccess ||
      nb < 1)
    nb = 1;
  cached.store(nb, std::memory_order_relaxed);
  return nb;
}

template <typename F, bool kPipe, bool kFull>
static hipError_t stretch_run(const StretchDev<F>& d, hipStream_t s) {
  constexpr int M = StretchShape<F>::M, KS = StretchShape<F>::KS;
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  // every resident wavefront slot, but no more wavefronts than tiles
  int64_t blocks = (int64_t)stretch_blocks_per_cu<F, kPipe, kFull>() * (ncu > 0 ? ncu : 1);
  const int64_t need = (d.total_tiles + 3) / 4;
  if (blocks > need) blocks = need;
  hipLaunchKernelGGL((stretch_kernel<F, M, KS, kPipe, kFull>), dim3((unsigned)blocks), dim3(256), 0, s,
                     d);
  return hipGetLastError();
}

template <typename F>
static hipError_t stretch_launch(const TileGeom& g, const StretchArgs& s_, hipStream_t s) {
  const int V = Vec<F>::n;
  StretchDev<F> d;
  d.u_start = (const F*)s_.u_start;
  d.lam_in = (const F*)s_.lam_in;
  d.lam_out = (F*)s_.lam_out;
  d.partials = s_.partials;
  d.N = s_.N;
  d.total_tiles = g.tiles_per_rod * s_.nrods;
  d.tiles_per_rod = g.tiles_per_rod;
  d.part_stride = s_.part_stride;
  d.part_off = s_.part_off;
  d.part_rods = s_.nrods;
  d.H = g.H;
  d.len = s_.len;
  d.r = (F)s_.r;
  d.c1 = (F)s_.c1;
  d.cN = (F)s_.cN;
  const bool al = is_aligned16(s_.u_start) && is_aligned16(s_.lam_in) && is_aligned16(s_.lam_out);
  d.aligned = al && (s_.nrods == 1 || s_.N % V == 0);
  if (d.total_tiles <= 0) return hipSuccess;
  const bool full = s_.len == StretchShape<F>::KS;
  const int64_t lim = (int64_t)1 << 31;
  const bool pipe = al && s_.N % V == 0 && s_.N >= g.L && d.total_tiles < lim &&
                    s_.N * (int64_t)sizeof(F) < lim && s_.part_stride * s_.nrods * 8 < lim;
  if (pipe) return full ? stretch_run<F, true, true>(d, s) : stretch_run<F, true, false>(d, s);
  return stretch_run<F, false, false>(d, s);
}

hipError_t launch_adjoint_stretch(int dtype, const TileGeom& g, const StretchArgs& a,
                                  hipStream_t s) {
  if (a.len < 1 || a.len > stretch_steps(dtype) || g.H < stretch_steps(dtype) + 1 ||
      g.tiles_per_rod <= 0 || a.part_off + g.tiles_per_rod > a.part_stride)
    return hipErrorInvalidValue;
  if (g.M != stretch_pts_per_lane(dtype)) return hipErrorInvalidValue;
  return dtype == 0 ? stretch_launch<float>(g, a, s) : stretch_launch<double>(g, a, s);
}

// grad_r[b] = sum of partials[b*n .. b*n + n).  Up to kChunk entries per rod
// one pass; beyond that each chunk's sum first replaces the chunk's first entry
// (a block reads only its own chunk, so nothing it overwrites is read by
// another block), then one more pass adds the chunk sums.
hipError_t launch_reduce_partials(double* partials, int64_t n, int64_t nrods, double* grad_r,
                                  hipStream_t s) {
  constexpr int64_t kChunk = 8192;
  const unsigned rods = (unsigned)(nrods > 0 ? nrods : 1);
  if (n <= kChunk) {
    hipLaunchKernelGGL(reduce_chunks_kernel, dim3(1, rods), dim3(256), 0, s,
                       (const double*)partials, n, n, (int64_t)1, kChunk, grad_r, (int64_t)1,
                       (int64_t)0);
    return hipGetLastError();
  }
  const int64_t nchunks = (n + kChunk - 1) / kChunk;
  hipLaunchKernelGGL(reduce_chunks_kernel, dim3((unsigned)nchunks, rods), dim3(256), 0, s,
                     (const double*)partials, n, n, (int64_t)1, kChunk, partials, n, kChunk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_chunks_kernel, dim3(1, rods), dim3(256), 0, s,
                     (const double*)partials, nchunks, n, kChunk, nchunks, grad_r, (int64_t)1,
                     (int64_t)0);
  return hipGetLastError();
}

}  // namespace heat1d
