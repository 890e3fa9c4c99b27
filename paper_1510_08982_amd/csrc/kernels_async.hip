// kernels_async.hip -- the asynchronous iteration of Eq.4 (Section 3) as one
// persistent kernel with no grid-wide barrier.
//
// Workgroup b owns subdomain p (Fig. 1: a PE owns a group of grid points) and
// keeps its points in registers for all K steps.  Inside the workgroup every
// read is current (Section 3: no asynchrony inside a PE): wavefronts trade
// their edge points through LDS behind one barrier per step.  Across
// workgroups, each subdomain publishes its first and last point after every
// step into a ring of Q = 2d+2 slots in global memory and then release-stores
// its progress counter; a neighbour acquire-polls that counter and reads the
// slot of the step it needs.  With staleness at most d, a writer can be at most
// d+1 steps ahead of a reader that still needs a slot, so 2d+2 slots never
// overwrite a value still in use (the buffer of length q of Eq.4, doubled for
// the writer's lead).
//
// Emulated mode reads exactly step max(0, k - delta(k,p,side)) of the seeded
// schedule; hardware mode reads the newest published step not newer than k and
// waits only while that step is older than k - d.
#include "heat1d_device.h"
#include "heat1d_launch.h"

namespace heat1d {

constexpr int kMaxStatDelay = 255;

struct AsyncDev {
  const void* in;
  void* out;
  int64_t N;
  int32_t P;
  int32_t K;
  int32_t d;
  int32_t Q;
  uint64_t seed;
  int32_t mode;
  int32_t remap;
  double r, c1, cN;
  void* ring;
  int32_t* prog;
  int32_t* err;
  int64_t* stats;
  int64_t watchdog;
};

__device__ __forceinline__ void ring_put(float* p, float v) {
  __hip_atomic_store(reinterpret_cast<uint32_t*>(p), __float_as_uint(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void ring_put(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<uint64_t*>(p), (uint64_t)__double_as_longlong(v),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ring_get(float* p) {
  return __uint_as_float(__hip_atomic_load(reinterpret_cast<uint32_t*>(p), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ double ring_get(double* p) {
  return __longlong_as_double((long long)__hip_atomic_load(
      reinterpret_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Wait until *flag >= need.  Returns the last value seen, or -1 if the watchdog
// expired or another workgroup aborted the run.
__device__ __forceinline__ int poll_flag(int32_t* flag, int need, int64_t watchdog, int32_t* err,
                                         unsigned long long* polls) {
  int64_t n = 0;
  for (;;) {
    const int v = uniform(__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT));
    if (v >= need) {
      *polls += (unsigned long long)n;
      return v;
    }
    ++n;
    if (n > watchdog) {
      if ((threadIdx.x & (kWave - 1)) == 0) {
        atomicCAS(err, 0, 4 /* HEAT1D_ETIMEOUT */);
        __hip_atomic_store(err + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      *polls += (unsigned long long)n;
      return -1;
    }
    if ((n & 63) == 0 &&
        uniform(__hip_atomic_load(err + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0) {
      *polls += (unsigned long long)n;
      return -1;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// Fetch the value a subdomain edge reads at step k from its neighbour's ring.
// Returns false on abort.
template <typename F, int kMode, bool kStats>
__device__ __forceinline__ bool fetch_halo(const AsyncDev& a, int k, int p, int side,
                                           int32_t* flag, F* ring, F* out,
                                           unsigned long long* s_stats) {
  int tstar, need;
  if constexpr (kMode == 0) {
    const int dl = delay_of(a.seed, k, p, side, a.P, a.d);
    tstar = k - dl > 0 ? k - dl : 0;
    need = tstar;
  } else {
    need = k - a.d > 0 ? k - a.d : 0;
    tstar = 0;
  }
  unsigned long long polls = 0;
  const int seen = poll_flag(flag, need, a.watchdog, a.err, &polls);
  if (seen < 0) return false;
  if constexpr (kMode != 0) tstar = seen < k ? seen : k;
  *out = ring_get(ring + (tstar % a.Q));
  if (kStats && (threadIdx.x & (kWave - 1)) == 0) {
    const int used = k - tstar;
    atomicAdd(&s_stats[used <= kMaxStatDelay ? used : kMaxStatDelay], 1ull);
    atomicAdd(&s_stats[kMaxStatDelay + 1], polls);
    atomicAdd(&s_stats[kMaxStatDelay + 2], 1ull);
  }
  return true;
}

template <typename F, int M, int kMode, bool kStats>
__global__ __launch_bounds__(1024) void async_kernel(const AsyncDev a) {
  __shared__ F lds[4 * 16];
  __shared__ int s_abort_at;
  __shared__ unsigned long long s_stats[kMaxStatDelay + 3];

  const int nw = blockDim.x / kWave;
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int b = blockIdx.x;
  const int P = a.P;
  const int p = a.remap ? ((b % 8) * (P / 8) + b / 8) : b;
  const int64_t lo = (int64_t)p * a.N / P;
  const int64_t hi = (int64_t)(p + 1) * a.N / P;
  const int S = (int)(hi - lo);
  const F r = (F)a.r, c1 = (F)a.c1, cN = (F)a.cN;
  const int Q = a.Q;

  for (int i = threadIdx.x; i < kMaxStatDelay + 3; i += blockDim.x) s_stats[i] = 0;
  if (threadIdx.x == 0) s_abort_at = 0x7fffffff;

  const F* __restrict__ src = reinterpret_cast<const F*>(a.in) + lo;
  F* __restrict__ dst = reinterpret_cast<F*>(a.out) + lo;
  F* ring = reinterpret_cast<F*>(a.ring);
  F* ringL = ring + (int64_t)(2 * p) * Q;      // this subdomain's first point
  F* ringR = ring + (int64_t)(2 * p + 1) * Q;  // this subdomain's last point
  int32_t* progL = a.prog + 2 * p;
  int32_t* progR = a.prog + 2 * p + 1;

  F u[M];
  const int q0 = (wave * kWave + lane) * M;
  load_points<F, M>(u, src, q0, S, false);

  // local position of the subdomain's last point
  const int rq = S - 1;
  const int rw = rq / (kWave * M);
  const int rl = (rq / M) % kWave;
  const int rj = uniform(rq % M);
  const bool active = wave * kWave * M < S;
  const bool has_left = p > 0;
  const bool has_right = p < P - 1;

  // Dirichlet ends (Section 2) at k = 0
  if (!has_left && wave == 0) u[0] = (lane == 0) ? c1 : u[0];
  if (!has_right && wave == rw) set_point<F, M>(u, rj, lane == rl, cN);

  // publish u(0)
  if (wave == 0 && has_left) {
    const F v = read_lane(u[0], 0);
    if (lane == 0) {
      ring_put(ringL, v);
      __hip_atomic_store(progL, 0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (wave == rw && has_right) {
    const F v = read_lane(get_point<F, M>(u, rj), rl);
    if (lane == 0) {
      ring_put(ringR, v);
      __hip_atomic_store(progR, 0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  __syncthreads();

  for (int k = 0; k < a.K; ++k) {
    F hl = F(0), hr = F(0);
    bool ok = true;
    if (wave == 0 && has_left)
      ok = fetch_halo<F, kMode, kStats>(a, k, p, 0, a.prog + 2 * (p - 1) + 1, ring + (int64_t)(2 * (p - 1) + 1) * Q,
                         &hl, s_stats);
    if (ok && wave == rw && has_right)
      ok = fetch_halo<F, kMode, kStats>(a, k, p, 1, a.prog + 2 * (p + 1), ring + (int64_t)(2 * (p + 1)) * Q, &hr,
                         s_stats);

    F left = from_lower_lane(u[M - 1]);
    F right = from_upper_lane(u[0]);
    if (nw > 1) {
      F* buf = lds + (k & 1) * 2 * nw;
      if (lane == 0) buf[2 * wave] = u[0];
      if (lane == kWave - 1) buf[2 * wave + 1] = u[M - 1];
      if (!ok && lane == 0) atomicMin(&s_abort_at, k);
      __syncthreads();
      if (s_abort_at <= k) break;
      const F lw = wave > 0 ? buf[2 * (wave - 1) + 1] : F(0);
      const F rw_ = wave + 1 < nw ? buf[2 * (wave + 1)] : F(0);
      left = (lane == 0) ? lw : left;
      right = (lane == kWave - 1) ? rw_ : right;
    } else if (!ok) {
      break;
    }
    if (!active) continue;

    if (wave == 0 && has_left) left = (lane == 0) ? hl : left;
    if (wave == rw && has_right) {
      if (rj == M - 1)
        right = (lane == rl) ? hr : right;
      else
        set_point<F, M>(u, rj + 1, lane == rl, hr);
    }
    lane_step<F, M>(u, left, right, r);
    if (!has_left && wave == 0) u[0] = (lane == 0) ? c1 : u[0];
    if (!has_right && wave == rw) set_point<F, M>(u, rj, lane == rl, cN);

    // publish u(k+1)
    const int slot = (k + 1) % Q;
    if (wave == 0 && has_left) {
      const F v = read_lane(u[0], 0);
      if (lane == 0) {
        ring_put(ringL + slot, v);
        __hip_atomic_store(progL, k + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (wave == rw && has_right) {
      const F v = read_lane(get_point<F, M>(u, rj), rl);
      if (lane == 0) {
        ring_put(ringR + slot, v);
        __hip_atomic_store(progR, k + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
  if (active) store_points<F, M>(u, dst, q0, q0, 0, S, false);

  if constexpr (kStats) {
    __syncthreads();
    const int nst = a.d + 3;
    for (int i = threadIdx.x; i < nst; i += blockDim.x) {
      unsigned long long v;
      if (i <= a.d) v = s_stats[i <= kMaxStatDelay ? i : kMaxStatDelay];
      else v = s_stats[kMaxStatDelay + 1 + (i - a.d - 1)];
      if (v) atomicAdd(reinterpret_cast<unsigned long long*>(a.stats) + i, v);
    }
  }
}

__global__ void async_prepare_kernel(int32_t* prog, int64_t n, int32_t* err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) prog[i] = -1;
  if (i < 2) err[i] = 0;
}

__global__ void delay_schedule_kernel(int32_t P, int64_t K, int32_t d, uint64_t seed,
                                      uint8_t* out) {
  const int64_t total = K * P * 2;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int side = (int)(i & 1);
    const int64_t kp = i >> 1;
    const int64_t k = kp / P;
    const int64_t p = kp - k * P;
    out[i] = (uint8_t)delay_of(seed, k, p, side, P, d);
  }
}

// ---------------------------------------------------------------------------
bool async_supports(int dtype, int M) {
  if (dtype == 0) return M == 1 || M == 2 || M == 4 || M == 8 || M == 16 || M == 32 || M == 64;
  return M == 1 || M == 2 || M == 4 || M == 8 || M == 16 || M == 32;
}

template <int kMode, bool kStats>
static const void* async_fn_t(int dtype, int M) {
#define HEAT1D_AF(FT, MM) \
  case MM:                \
    return reinterpret_cast<const void*>(&async_kernel<FT, MM, kMode, kStats>);
  if (dtype == 0) {
    switch (M) {
      HEAT1D_AF(float, 1)
      HEAT1D_AF(float, 2)
      HEAT1D_AF(float, 4)
      HEAT1D_AF(float, 8)
      HEAT1D_AF(float, 16)
      HEAT1D_AF(float, 32)
      HEAT1D_AF(float, 64)
    }
  } else {
    switch (M) {
      HEAT1D_AF(double, 1)
      HEAT1D_AF(double, 2)
      HEAT1D_AF(double, 4)
      HEAT1D_AF(double, 8)
      HEAT1D_AF(double, 16)
      HEAT1D_AF(double, 32)
    }
  }
#undef HEAT1D_AF
  return nullptr;
}

static const void* async_fn(int dtype, int M, int mode, bool stats) {
  if (mode == 0) return stats ? async_fn_t<0, true>(dtype, M) : async_fn_t<0, false>(dtype, M);
  return stats ? async_fn_t<1, true>(dtype, M) : async_fn_t<1, false>(dtype, M);
}

int async_max_resident_groups(int dtype, int M, int waves, int /*Q*/) {
  const void* fn = async_fn(dtype, M, 1, true);
  if (!fn) return 0;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, waves * kWave, 0) != hipSuccess)
    return 0;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return per_cu * ncu;
}

hipError_t launch_async_prepare(const AsyncLaunch& a, hipStream_t s) {
  const int64_t n = (int64_t)a.P * 2;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(async_prepare_kernel, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0,
                     s, a.prog, n, a.err);
  return hipGetLastError();
}

hipError_t launch_async(const AsyncLaunch& a, hipStream_t s) {
  const void* fn = async_fn(a.dtype, a.M, a.mode, a.stats != nullptr);
  if (!fn) return hipErrorInvalidValue;
  AsyncDev d;
  d.in = a.in;
  d.out = a.out;
  d.N = a.N;
  d.P = a.P;
  d.K = a.K;
  d.d = a.d;
  d.Q = a.Q;
  d.seed = a.seed;
  d.mode = a.mode;
  d.remap = a.remap;
  d.r = a.r;
  d.c1 = a.c1;
  d.cN = a.cN;
  d.ring = a.ring;
  d.prog = a.prog;
  d.err = a.err;
  d.stats = a.stats;
  d.watchdog = a.watchdog;
  void* args[] = {&d};
  return hipLaunchCooperativeKernel(fn, dim3((unsigned)a.P), dim3((unsigned)(a.waves * kWave)),
                                    args, 0, s);
}

hipError_t launch_delay_schedule(int32_t P, int64_t K, int32_t d, uint64_t seed, uint8_t* out,
                                 hipStream_t s) {
  const int64_t total = K * P * 2;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65535) blocks = 65535;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(delay_schedule_kernel, dim3((unsigned)blocks), dim3(256), 0, s, P, K, d, seed,
                     out);
  return hipGetLastError();
}

}  // namespace heat1d
