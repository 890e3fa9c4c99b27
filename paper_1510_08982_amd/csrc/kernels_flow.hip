// kernels_flow.hip -- every pass of the temporally blocked synchronous
// iteration (Eq.3, Section 2) in one persistent launch, ordered by the data
// each tile needs instead of by a barrier after each pass.
//
// Item k of the launch is tile i = k mod ntiles of pass p = k div ntiles, in
// the tile geometry of the tiled kernel (pass p advances steps pT .. pT+T-1).
// Wavefront w of W takes items w, w+W, w+2W, ... in order.  Tile i of pass p
// reads the window of the state after pass p-1 that tiles i-1, i, i+1 of pass
// p-1 wrote, and overwrites (in the other buffer of the ping-pong pair) the
// points those same three tiles read for pass p-1: so the one condition
// "tiles i-1, i, i+1 of the rod have finished pass p-1" covers both the values
// it reads and the values it overwrites.  done[i] holds the last pass tile i
// has finished; it is set after the tile's stores have completed (deferred
// until the wavefront's next tile has issued its loads).  The state is
// written and (from pass 1 on) read with 64-bit agent-scope relaxed atomics,
// which reach the device coherence point, so no cache write-back or
// invalidation is ever needed between CUs on different XCDs.
//
// Progress: every item waits only for items with smaller k.  The wavefront
// holding the smallest unfinished item never waits on an unfinished item (each
// wavefront takes its items in increasing order, so any smaller item is done or
// held by a wavefront that is at it), provided all W wavefronts are resident:
// the launch is cooperative, which guarantees that or fails.  A pass thus
// starts on the tiles whose inputs are ready while the previous pass is still
// finishing elsewhere, and a run pays one launch and one tail instead of one
// per pass.  Every wait is bounded by a watchdog that records HEAT1D_ETIMEOUT
// and raises an abort flag.
#include "heat1d_device.h"
#include "heat1d_launch.h"
#include "heat1d_steps.h"

#include <atomic>

namespace heat1d {

template <typename F>
struct FlowDev {
  const F* u0;
  F* uK;
  F* ws;
  int64_t N;
  int64_t nrods;
  int64_t tiles_per_rod;
  int H;
  int T;
  int K;
  int passes;
  F r, c1, cN;
  StepWeights<F> sw;
  int32_t* done;  // [nrods * tiles_per_rod]: last pass finished, -1 before the first
  int32_t* err;   // [0] status, [1] abort flag
  int64_t watchdog;
};

// Whether the tiles j0 .. j1 (at most three) have finished pass `need`: the
// counters are read in one round trip.
template <typename F>
__device__ __forceinline__ bool deps_ready(const FlowDev<F>& a, int64_t j0, int64_t j1, int need) {
  int v = INT32_MAX;
  for (int64_t j = j0; j <= j1; ++j) {
    const int x = __hip_atomic_load(a.done + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    v = x < v ? x : v;
  }
  return uniform(v) >= need;
}

// Wait until the tiles j0 .. j1 have finished pass `need`.  False if the
// watchdog expired or the run was aborted.
template <typename F>
__device__ __forceinline__ bool wait_done(const FlowDev<F>& a, int64_t j0, int64_t j1, int need) {
  int64_t n = 0;
  for (;;) {
    if (deps_ready(a, j0, j1, need)) return true;
    ++n;
    if (n > a.watchdog) {
      if ((threadIdx.x & (kWave - 1)) == 0) {
        atomicCAS(a.err, 0, 4 /* HEAT1D_ETIMEOUT */);
        __hip_atomic_store(a.err + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      return false;
    }
    if ((n & 63) == 0 &&
        uniform(__hip_atomic_load(a.err + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0)
      return false;
    __builtin_amdgcn_s_sleep(1);
  }
}

// A finished tile's pass number is published only once its stores have
// completed.  Waiting for that right after the stores would stall the
// wavefront for the write-through latency of every tile, so the publication
// is deferred: it happens after the next tile's loads are issued (so the wait
// covers only the older stores), before the wavefront would block on a
// dependence, or at the end of its work.
template <typename F>
__device__ __forceinline__ void publish(const FlowDev<F>& a, int64_t i, int p, int lane) {
  if (i >= 0 && lane == 0)
    __hip_atomic_store(a.done + i, p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename F, int M, int S>
__global__ __launch_bounds__(256) void flow_kernel(const FlowDev<F> a) {
  constexpr int L = kWave * M;
  constexpr int kLoads = M / WordPts<F>::n;  // memory instructions of one tile load
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t W = (int64_t)gridDim.x * (blockDim.x / kWave);
  const int64_t tpr = a.tiles_per_rod;
  const int64_t ntiles = tpr * a.nrods;
  const int64_t total = (int64_t)a.passes * ntiles;
  const int Wout = L - 2 * a.H;
  int64_t prev_i = -1;  // tile whose pass number is not yet published
  int prev_p = 0;
  for (int64_t k = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; k < total;
       k += W) {
    const int p = (int)(k / ntiles);
    const int64_t i = k - (int64_t)p * ntiles;
    const int64_t rod = i / tpr;
    const int64_t t = i - rod * tpr;
    const int steps = a.K - p * a.T < a.T ? a.K - p * a.T : a.T;
    // the ping-pong pair is arranged so that the last pass writes uK
    const F* in = p == 0 ? a.u0 : (((a.passes - p) % 2 == 0) ? a.uK : a.ws);
    F* out = ((a.passes - 1 - p) % 2 == 0) ? a.uK : a.ws;
    const int64_t g0 = t * Wout + lane * M;
    if (p > 0) {
      const int64_t j0 = t > 0 ? i - 1 : i;
      const int64_t j1 = t + 1 < tpr ? i + 1 : i;
      if (!deps_ready(a, j0, j1, p - 1)) {
        // about to block: publish the previous tile first, so that no
        // wavefront ever waits while holding an unpublished tile (the order
        // argument above then guarantees progress)
        if (prev_i >= 0) {
          asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
          publish(a, prev_i, prev_p, lane);
          prev_i = -1;
        }
        if (!wait_done(a, j0, j1, p - 1)) return;
      }
    }
    // one load path for every pass (u0 itself is never written, so the
    // coherent loads only cost it the L2 on the first pass)
    F u[M];
    if (t * Wout + L <= a.N) {
      // the whole tile lies inside the rod: every lane issues exactly kLoads
      // loads, so waiting until at most kLoads are outstanding leaves only
      // them, and everything older (the previous tile's stores) has completed
      load_coherent<F, M>(u, in + rod * a.N, g0, a.N);
      if (prev_i >= 0) {
        asm volatile("s_waitcnt vmcnt(%0)" ::"n"(kLoads) : "memory");
        publish(a, prev_i, prev_p, lane);
      }
    } else {
      // the rod's last tile: lanes past the end skip loads, so wait for all
      load_coherent<F, M>(u, in + rod * a.N, g0, a.N);
      if (prev_i >= 0) {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        publish(a, prev_i, prev_p, lane);
      }
    }
    tile_pass<F, M, S, true>(u, out + rod * a.N, a.N, t, tpr, a.H, steps, a.r, a.c1, a.cN, a.sw,
                             true, lane);
    prev_i = i;
    prev_p = p;
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  publish(a, prev_i, prev_p, lane);
}

// ---------------------------------------------------------------------------
static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

bool flow_applies(int dtype, const TileGeom& g, const void* u0, const void* uK, const void* ws,
                  int64_t N, int64_t max_tiles) {
  const int V = dtype == 0 ? 4 : 2;
  return aligned16(u0) && aligned16(uK) && aligned16(ws) && N % V == 0 && g.tiles_per_rod >= 1 &&
         g.tiles_per_rod <= max_tiles && 4 * g.H <= g.L;
}

template <typename F, int M, int S>
static int flow_blocks_per_cu() {
  static std::atomic<int> cached{0};
  int nb = cached.load(std::memory_order_relaxed);
  if (nb > 0) return nb;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, flow_kernel<F, M, S>, 256, 0) !=
          hipSuccess ||
      nb < 1)
    nb = 0;
  cached.store(nb, std::memory_order_relaxed);
  return nb;
}

template <typename F, int M, int S>
static hipError_t flow_launch(const FlowLaunch& f, hipStream_t s) {
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int per_cu = flow_blocks_per_cu<F, M, S>();
  if (per_cu < 1 || ncu < 1) return hipErrorLaunchOutOfResources;
  const int64_t ntiles = f.g.tiles_per_rod * f.nrods;
  int64_t blocks = (int64_t)per_cu * ncu;
  if (blocks * 4 > ntiles) blocks = (ntiles + 3) / 4;
  FlowDev<F> d;
  d.u0 = reinterpret_cast<const F*>(f.u0);
  d.uK = reinterpret_cast<F*>(f.uK);
  d.ws = reinterpret_cast<F*>(f.ws);
  d.N = f.N;
  d.nrods = f.nrods;
  d.tiles_per_rod = f.g.tiles_per_rod;
  d.H = f.g.H;
  d.T = f.T;
  d.K = f.K;
  d.passes = (f.K + f.T - 1) / f.T;
  d.r = (F)f.r;
  d.c1 = (F)f.c1;
  d.cN = (F)f.cN;
  d.sw = step_weights<F>(f.r, S);
  d.done = f.done;
  d.err = f.err;
  d.watchdog = f.watchdog;
  e = launch_fill_i32(f.done, -1, ntiles, s);
  if (e == hipSuccess) e = launch_fill_i32(f.err, 0, 2, s);
  if (e != hipSuccess) return e;
  void* args[] = {&d};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(flow_kernel<F, M, S>),
                                    dim3((unsigned)blocks), dim3(256), args, 0, s);
}

hipError_t launch_sync_flow(const FlowLaunch& f, hipStream_t s) {
  if (f.K < 1 || f.T < 1 || f.T > f.g.H || f.g.tiles_per_rod <= 0 ||
      !fused_supports(f.dtype, f.g.M, f.fuse))
    return hipErrorInvalidValue;
#define HEAT1D_FLOW(FT, MM, SS) \
  case (MM) * 8 + (SS):         \
    return flow_launch<FT, MM, SS>(f, s);
  if (f.dtype == 0) {
    switch (f.g.M * 8 + f.fuse) {
      HEAT1D_FOR_EACH_F32(HEAT1D_FLOW)
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (f.g.M * 8 + f.fuse) {
      HEAT1D_FOR_EACH_F64(HEAT1D_FLOW)
      default: return hipErrorInvalidValue;
    }
  }
#undef HEAT1D_FLOW
}

}  // namespace heat1d
