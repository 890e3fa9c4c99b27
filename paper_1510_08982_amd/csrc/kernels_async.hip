// kernels_async.hip -- the asynchronous iteration of Eq.4 (Section 3) as one
// persistent kernel with no grid-wide barrier.
//
// Workgroup b owns subdomain p (Fig. 1: a PE owns a group of grid points) and
// keeps its points in registers for all K steps.  Inside the workgroup every
// read is current (Section 3: no asynchrony inside a PE): wavefronts trade
// their edge points through LDS behind one barrier per step.  Across
// workgroups, each subdomain publishes its first and last point after every
// step into a ring of Q = 2d+2 slots in global memory; a neighbour reads the
// slot of the step it needs.  With staleness at most d, a writer can be at most
// d+1 steps ahead of a reader that still needs a slot, so 2d+2 slots never
// overwrite a value still in use (the buffer of length q of Eq.4, doubled for
// the writer's lead).
//
// A slot is a 64-bit word holding the step number in its upper half and the
// value (FP32, or one half of an FP64 value in each of two words) in its lower
// half, written and read with relaxed agent-scope atomics.  A reader accepts a
// slot only when its tag is the step it wants, so the single-copy atomicity of
// the word replaces any ordering between a data store and a flag store: no
// release/acquire fence, hence no L2 write-back or invalidate, is ever issued.
//
// Emulated mode reads exactly step max(0, k - delta(k,p,side)) of the seeded
// schedule; hardware mode reads the newest step the neighbour has announced
// (a relaxed hint word), never newer than k, and waits only while that step is
// older than k - d.
#include "heat1d_delays.h"
#include "heat1d_device.h"
#include "heat1d_launch.h"

#include <mutex>

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
  uint64_t* ring;  // [P][2][Q][words]
  int32_t* hint;   // [P][2]: newest step published (hardware mode)
  int32_t* err;    // [0] status, [1] abort flag
  int64_t* stats;
  int64_t watchdog;
  int32_t jitter;
  int32_t periodic;  // 1: the rod is a ring and subdomains 0 and P-1 are neighbours
  int32_t sched;     // emulated mode: the delay schedule
};

template <typename F> struct SlotWords;
template <> struct SlotWords<float> { static constexpr int n = 1; };
template <> struct SlotWords<double> { static constexpr int n = 2; };

__device__ __forceinline__ void put_word(uint64_t* p, uint32_t tag, uint32_t payload) {
  __hip_atomic_store(p, ((uint64_t)tag << 32) | payload, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
// The word as the whole wavefront sees it (all lanes read the same address).
__device__ __forceinline__ uint64_t get_word(uint64_t* p) {
  const uint64_t w = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t lo = (uint32_t)uniform((int)(uint32_t)w);
  const uint32_t hi = (uint32_t)uniform((int)(uint32_t)(w >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ void slot_put(uint64_t* s, int step, float v) {
  put_word(s, (uint32_t)step, __float_as_uint(v));
}
__device__ __forceinline__ void slot_put(uint64_t* s, int step, double v) {
  put_word(s, (uint32_t)step, (uint32_t)__double2loint(v));
  put_word(s + 1, (uint32_t)step, (uint32_t)__double2hiint(v));
}
// True when the slot holds step `step`; then *v is the value published for it.
__device__ __forceinline__ bool slot_get(uint64_t* s, int step, float* v) {
  const uint64_t w = get_word(s);
  if ((uint32_t)(w >> 32) != (uint32_t)step) return false;
  *v = __uint_as_float((uint32_t)w);
  return true;
}
__device__ __forceinline__ bool slot_get(uint64_t* s, int step, double* v) {
  const uint64_t w0 = get_word(s);
  const uint64_t w1 = get_word(s + 1);
  if ((uint32_t)(w0 >> 32) != (uint32_t)step || (uint32_t)(w1 >> 32) != (uint32_t)step)
    return false;
  *v = __hiloint2double((int)(uint32_t)w1, (int)(uint32_t)w0);
  return true;
}

// Fetch the value a subdomain edge reads at step k from its neighbour's ring
// (nring: the neighbour's edge ring, nhint: its newest-step hint).  Returns
// false if the watchdog expired or another workgroup aborted the run.
template <typename F, int kMode, bool kStats>
__device__ __forceinline__ bool fetch_halo(const AsyncDev& a, int k, int p, int side,
                                           uint64_t* nring, int32_t* nhint, F* out,
                                           unsigned long long* s_stats) {
  constexpr int W = SlotWords<F>::n;
  const int Q = a.Q;
  int tstar = 0;
  int64_t n = 0;
  if constexpr (kMode == 0) {
    const int dl = sched_delay(a.sched, a.seed, k, p, side, a.P, a.d);
    tstar = k - dl > 0 ? k - dl : 0;
  }
  const int lo = k - a.d > 0 ? k - a.d : 0;
  for (;;) {
    if constexpr (kMode == 0) {
      if (slot_get(nring + (int64_t)(tstar % Q) * W, tstar, out)) break;
    } else {
      const int h = uniform(__hip_atomic_load(nhint, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      tstar = h < k ? h : k;
      if (tstar >= lo && slot_get(nring + (int64_t)(tstar % Q) * W, tstar, out)) break;
    }
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
  if (kStats && (threadIdx.x & (kWave - 1)) == 0) {
    const int used = k - tstar;
    atomicAdd(&s_stats[used <= kMaxStatDelay ? used : kMaxStatDelay], 1ull);
    atomicAdd(&s_stats[kMaxStatDelay + 1], (unsigned long long)n);
    atomicAdd(&s_stats[kMaxStatDelay + 2], 1ull);
  }
  return true;
}

// Halo words read ahead of use: the loads for step k+1 are issued before the
// workgroup computes step k and are only inspected when step k+1 begins, so
// their latency overlaps the computation.  Emulated mode reads the slot of the
// scheduled step; hardware mode reads the slots of steps k+1 and k and keeps the
// newest one that has arrived.  A miss falls back to polling (fetch_halo).
template <typename F, int kMode>
struct HaloAhead {
  static constexpr int W = SlotWords<F>::n;
  uint64_t w[kMode == 0 ? W : 2 * W];
  int t;  // emulated: the step to read; hardware: the newest step wanted
};

template <typename F, int kMode>
__device__ __forceinline__ void ahead_issue(const AsyncDev& a, int k1, int p, int side,
                                            uint64_t* nring, HaloAhead<F, kMode>& h) {
  constexpr int W = SlotWords<F>::n;
  if constexpr (kMode == 0) {
    const int dl = sched_delay(a.sched, a.seed, k1, p, side, a.P, a.d);
    h.t = k1 - dl > 0 ? k1 - dl : 0;
    uint64_t* sl = nring + (int64_t)(h.t % a.Q) * W;
#pragma unroll
    for (int i = 0; i < W; ++i)
      h.w[i] = __hip_atomic_load(sl + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    h.t = k1;
    const int k0 = k1 > 0 ? k1 - 1 : 0;
    uint64_t* s1 = nring + (int64_t)(k1 % a.Q) * W;
    uint64_t* s0 = nring + (int64_t)(k0 % a.Q) * W;
#pragma unroll
    for (int i = 0; i < W; ++i) {
      h.w[i] = __hip_atomic_load(s1 + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      h.w[W + i] = __hip_atomic_load(s0 + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

__device__ __forceinline__ bool decode(const uint64_t* w, int step, float* v) {
  const uint32_t tag = (uint32_t)uniform((int)(uint32_t)(w[0] >> 32));
  if (tag != (uint32_t)step) return false;
  *v = __uint_as_float((uint32_t)uniform((int)(uint32_t)w[0]));
  return true;
}
__device__ __forceinline__ bool decode(const uint64_t* w, int step, double* v) {
  const uint32_t t0 = (uint32_t)uniform((int)(uint32_t)(w[0] >> 32));
  const uint32_t t1 = (uint32_t)uniform((int)(uint32_t)(w[1] >> 32));
  if (t0 != (uint32_t)step || t1 != (uint32_t)step) return false;
  *v = __hiloint2double(uniform((int)(uint32_t)w[1]), uniform((int)(uint32_t)w[0]));
  return true;
}

// The halo value for step k: from the words read ahead when they hold an
// acceptable step, else by polling.
template <typename F, int kMode, bool kStats>
__device__ __forceinline__ bool halo_resolve(const AsyncDev& a, int k, int p, int side,
                                             uint64_t* nring, int32_t* nhint,
                                             const HaloAhead<F, kMode>& h, F* out,
                                             unsigned long long* s_stats) {
  constexpr int W = SlotWords<F>::n;
  int used = -1;
  if constexpr (kMode == 0) {
    if (decode(h.w, h.t, out)) used = h.t;
  } else {
    const int lo = k - a.d > 0 ? k - a.d : 0;
    if (decode(h.w, k, out))
      used = k;
    else if (k >= 1 && k - 1 >= lo && decode(h.w + W, k - 1, out))
      used = k - 1;
  }
  if (used < 0) return fetch_halo<F, kMode, kStats>(a, k, p, side, nring, nhint, out, s_stats);
  if (kStats && (threadIdx.x & (kWave - 1)) == 0) {
    atomicAdd(&s_stats[k - used <= kMaxStatDelay ? k - used : kMaxStatDelay], 1ull);
    atomicAdd(&s_stats[kMaxStatDelay + 2], 1ull);
  }
  return true;
}

// kRagged: some subdomain's last point is not the last register of lane 63 of
// its last wavefront (N not a multiple of P, or N/P not the block's capacity).
// Without that case the right edge sits in a fixed register and the kernel
// carries no register-indexed writes or reads of it.
template <typename F, int M, int kMode, bool kStats, bool kRagged>
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
  constexpr int SW = SlotWords<F>::n;
  uint64_t* ringL = a.ring + (int64_t)(2 * p) * Q * SW;      // this subdomain's first point
  uint64_t* ringR = a.ring + (int64_t)(2 * p + 1) * Q * SW;  // this subdomain's last point
  int32_t* hintL = a.hint + 2 * p;
  int32_t* hintR = a.hint + 2 * p + 1;

  F u[M];
  const int q0 = (wave * kWave + lane) * M;
  load_points<F, M>(u, src, q0, S, false);

  // local position of the subdomain's last point
  const int rq = S - 1;
  const int rw = rq / (kWave * M);
  const int rl = (rq / M) % kWave;
  const int rj = kRagged ? uniform(rq % M) : M - 1;
  const bool active = wave * kWave * M < S;
  // On the ring of Section 5.3 (P >= 2) every subdomain has two neighbours:
  // subdomain 0 reads the last point of P-1 and P-1 reads the first point of 0.
  const bool ring = a.periodic != 0;
  const bool has_left = p > 0 || ring;
  const bool has_right = p < P - 1 || ring;
  const int pl = p > 0 ? p - 1 : P - 1;
  const int pr = p < P - 1 ? p + 1 : 0;

  // Dirichlet ends (Section 2) at k = 0
  if (!has_left && wave == 0) u[0] = (lane == 0) ? c1 : u[0];
  if (!has_right && wave == rw) {
    if constexpr (kRagged)
      set_point<F, M>(u, rj, lane == rl, cN);
    else
      u[M - 1] = (lane == rl) ? cN : u[M - 1];
  }

  // publish u(0)
  if (wave == 0 && has_left) {
    const F v = read_lane(u[0], 0);
    if (lane == 0) {
      slot_put(ringL, 0, v);
      if (kMode != 0) __hip_atomic_store(hintL, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (wave == rw && has_right) {
    const F v = read_lane(kRagged ? get_point<F, M>(u, rj) : u[M - 1], rl);
    if (lane == 0) {
      slot_put(ringR, 0, v);
      if (kMode != 0) __hip_atomic_store(hintR, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  __syncthreads();

  // neighbour rings: the last point of the left neighbour and the first point
  // of the right one
  uint64_t* nringL = has_left ? a.ring + (int64_t)(2 * pl + 1) * Q * SW : a.ring;
  uint64_t* nringR = has_right ? a.ring + (int64_t)(2 * pr) * Q * SW : a.ring;
  int32_t* nhintL = has_left ? a.hint + 2 * pl + 1 : a.hint;
  int32_t* nhintR = has_right ? a.hint + 2 * pr : a.hint;
  HaloAhead<F, kMode> aheadL, aheadR;
  if (a.K > 0) {
    if (wave == 0 && has_left) ahead_issue<F, kMode>(a, 0, p, 0, nringL, aheadL);
    if (wave == rw && has_right) ahead_issue<F, kMode>(a, 0, p, 1, nringR, aheadR);
  }

  for (int k = 0; k < a.K; ++k) {
    F hl = F(0), hr = F(0);
    bool ok = true;
    if (wave == 0 && has_left)
      ok = halo_resolve<F, kMode, kStats>(a, k, p, 0, nringL, nhintL, aheadL, &hl, s_stats);
    if (ok && wave == rw && has_right)
      ok = halo_resolve<F, kMode, kStats>(a, k, p, 1, nringR, nhintR, aheadR, &hr, s_stats);

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

    if (a.jitter > 0) {
      // a seeded pause (the other wavefronts meet this one at the next barrier)
      const uint64_t h = sm64(a.seed ^ sm64(((uint64_t)k << 24) ^ (uint64_t)p ^ 0x5bd1e995ull));
      const int n = uniform((int)((h >> 33) % (uint64_t)(a.jitter + 1)));
      for (int i = 0; i < n; ++i) __builtin_amdgcn_s_sleep(1);
    }

    // read step k+1's halo words now; they are inspected after this step
    if (k + 1 < a.K) {
      if (wave == 0 && has_left) ahead_issue<F, kMode>(a, k + 1, p, 0, nringL, aheadL);
      if (wave == rw && has_right) ahead_issue<F, kMode>(a, k + 1, p, 1, nringR, aheadR);
    }

    if (wave == 0 && has_left) left = (lane == 0) ? hl : left;
    if (wave == rw && has_right) {
      if (!kRagged || rj == M - 1)
        right = (lane == rl) ? hr : right;
      else
        set_point<F, M>(u, rj + 1, lane == rl, hr);
    }
    lane_step<F, M>(u, left, right, r);
    if (!has_left && wave == 0) u[0] = (lane == 0) ? c1 : u[0];
    if (!has_right && wave == rw) {
      if constexpr (kRagged)
        set_point<F, M>(u, rj, lane == rl, cN);
      else
        u[M - 1] = (lane == rl) ? cN : u[M - 1];
    }

    // publish u(k+1)
    const int64_t slot = (int64_t)((k + 1) % Q) * SW;
    if (wave == 0 && has_left) {
      const F v = read_lane(u[0], 0);
      if (lane == 0) {
        slot_put(ringL + slot, k + 1, v);
        if (kMode != 0)
          __hip_atomic_store(hintL, k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (wave == rw && has_right) {
      // the last point sits in the last register unless the subdomain is ragged
      const F v = read_lane((!kRagged || rj == M - 1) ? u[M - 1] : get_point<F, M>(u, rj), rl);
      if (lane == 0) {
        slot_put(ringR + slot, k + 1, v);
        if (kMode != 0)
          __hip_atomic_store(hintR, k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

__global__ void async_prepare_kernel(uint64_t* ring, int64_t nwords, int32_t* hint, int64_t nhint,
                                     int32_t* err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += stride)
    ring[i] = ~0ull;  // tag 0xffffffff: no step published yet
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nhint; i += stride)
    hint[i] = -1;
  if (blockIdx.x == 0 && threadIdx.x < 2) err[threadIdx.x] = 0;
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

template <int kMode, bool kStats, bool kRagged>
static const void* async_fn_t(int dtype, int M) {
#define HEAT1D_AF(FT, MM) \
  case MM:                \
    return reinterpret_cast<const void*>(&async_kernel<FT, MM, kMode, kStats, kRagged>);
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

static const void* async_fn(int dtype, int M, int mode, bool stats, bool ragged) {
  if (ragged) {
    if (mode == 0)
      return stats ? async_fn_t<0, true, true>(dtype, M) : async_fn_t<0, false, true>(dtype, M);
    return stats ? async_fn_t<1, true, true>(dtype, M) : async_fn_t<1, false, true>(dtype, M);
  }
  if (mode == 0)
    return stats ? async_fn_t<0, true, false>(dtype, M) : async_fn_t<0, false, false>(dtype, M);
  return stats ? async_fn_t<1, true, false>(dtype, M) : async_fn_t<1, false, false>(dtype, M);
}

// Whether some subdomain ends short of its block's last register (kRagged).
static bool async_ragged(int64_t N, int32_t P, int M, int waves) {
  return N % P != 0 || N / P != (int64_t)waves * kWave * M;
}

int async_max_resident_groups(int dtype, int M, int waves, int /*Q*/) {
  const void* fn = async_fn(dtype, M, 1, true, true);
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

// ---------------------------------------------------------------------------
// Fixed scratch of the allocation-free run (heat1d_run_async_noalloc): the
// halo ring, the progress hints and the two status words of one run live in
// this array instead of a caller's workspace.  Each device that runs the
// library holds its own copy until the process ends.  Host code never passes
// the array's name to a kernel (on the host it only names the symbol): the
// device address comes from hipGetSymbolAddress, once per device, with that
// device current, and is kept per device.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t async_noalloc_scratch(void** ptr) {
  *ptr = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

__global__ void copy_status_kernel(const int32_t* err, int32_t* status) {
  if (threadIdx.x == 0) *status = *err;
}

hipError_t launch_copy_status(const int32_t* err, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(copy_status_kernel, dim3(1), dim3(64), 0, s, err, status);
  return hipGetLastError();
}

hipError_t launch_async_prepare(const AsyncLaunch& a, hipStream_t s) {
  const int64_t words = (int64_t)a.P * 2 * a.Q * (a.dtype == 0 ? 1 : 2);
  int64_t blocks = (words + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(async_prepare_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     reinterpret_cast<uint64_t*>(a.ring), words, a.prog, (int64_t)a.P * 2, a.err);
  return hipGetLastError();
}

hipError_t launch_async(const AsyncLaunch& a, hipStream_t s) {
  const void* fn =
      async_fn(a.dtype, a.M, a.mode, a.stats != nullptr, async_ragged(a.N, a.P, a.M, a.waves));
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
  d.ring = reinterpret_cast<uint64_t*>(a.ring);
  d.hint = a.prog;
  d.err = a.err;
  d.stats = a.stats;
  d.watchdog = a.watchdog;
  d.jitter = a.jitter;
  d.periodic = a.periodic;
  d.sched = a.sched;
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
