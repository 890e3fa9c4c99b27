// kernels_batched.hip -- thousands of independent rods of uneven length, step
// count and r in one persistent launch.
//
// One workgroup of 16 wavefronts runs per compute unit and keeps each rod it
// works on resident in registers for all of the rod's K steps.  Rods are
// grouped by length so that every lane holds enough points to amortise the
// per-step exchange:
//   phase 1  rods longer than a 4-wavefront group holds run on the whole
//            workgroup (edge exchange through LDS behind s_barrier);
//   phase 2  the workgroup splits into 4 groups of 4 wavefronts; each group
//            takes rods of medium length on its own, synchronised by an LDS
//            arrival counter;
//   phase 3  once the medium queue is empty, every wavefront takes short rods
//            alone, with DPP lane exchange only and no barrier at all.
// Each queue is ordered longest N*K first.  A rod of a small queue runs its K
// steps one after the other on few wavefronts, so its time, not its work, can
// set the end of the launch if it starts late: the first `small_first`
// workgroups therefore take the group and wavefront queues first and the
// whole-workgroup queue last, the others the reverse, and the queues are
// shared, so whichever empties first hands its workgroups to the rest.  The points-per-lane count M of a rod is the smallest
// instantiated value that holds it.
#include "heat1d_device.h"
#include "heat1d_launch.h"
#include "heat1d_rod.h"

namespace heat1d {

constexpr int kBatchWaves = 16;
constexpr int kGroupWaves = 4;
constexpr int kGroups = kBatchWaves / kGroupWaves;

template <typename F>
struct BatchDev {
  const F* in;
  F* out;
  const int64_t* offsets;
  const double* r;
  const double* c1;
  const double* cN;
  const int32_t* K;
  const int32_t* order[3];  // whole-workgroup, group and wavefront rods, longest first
  int32_t count[3];
  int32_t* heads;           // three queue counters
  int32_t small_first;      // workgroups that start with the group and wavefront queues
};

// Smallest supported M with capacity >= n for a block of `lanes` lanes.  The
// steps between instantiated counts are at most a third of the count above 6,
// so a rod's block computes at most a fifth more points than the rod holds
// (about 9 % over the benchmark's batch, where steps of a half cost 18 %).
__device__ __forceinline__ int pick_m(int n, int lanes) {
  const int need = (n + lanes - 1) / lanes;
  if (need <= 4) return 4;
  if (need <= 6) return 6;
  if (need <= 8) return 8;
  if (need <= 10) return 10;
  if (need <= 12) return 12;
  if (need <= 14) return 14;
  if (need <= 16) return 16;
  if (need <= 20) return 20;
  if (need <= 24) return 24;
  if (need <= 28) return 28;
  if (need <= 32) return 32;
  if (need <= 40) return 40;
  if (need <= 48) return 48;
  if (need <= 56) return 56;
  return 64;
}

template <typename F, RodSync kSync>
__device__ __forceinline__ void run_one(const BatchDev<F>& b, int rod, F* lds, int nwaves,
                                        int wave, int lane, int* count, int* epoch) {
  const int64_t off = b.offsets[rod];
  const int n = (int)(b.offsets[rod + 1] - off);
  const F r = (F)b.r[rod], c1 = (F)b.c1[rod], cN = (F)b.cN[rod];
  const int K = b.K[rod];
  const F* src = b.in + off;
  F* dst = b.out + off;
  const int m = uniform(pick_m(n, nwaves * kWave));
#define HEAT1D_RUN(MM)                                                                  \
  case MM:                                                                              \
    rod_resident<F, MM, kSync>(src, dst, n, K, r, c1, cN, lds, nwaves, wave, lane, false, \
                               count, epoch);                                           \
    break;
  // group and wavefront rods hold at most 128 bytes per lane (their queues are
  // filled that way), so only whole-workgroup rods instantiate the larger M
  constexpr bool kLarge = kSync == RodSync::kWorkgroup;
  switch (m) {
    HEAT1D_RUN(4)
    HEAT1D_RUN(6)
    HEAT1D_RUN(8)
    HEAT1D_RUN(10)
    HEAT1D_RUN(12)
    HEAT1D_RUN(14)
    HEAT1D_RUN(16)
    default:
      if constexpr (sizeof(F) == 4 || kLarge) {
        switch (m) {
          HEAT1D_RUN(20)
          HEAT1D_RUN(24)
          HEAT1D_RUN(28)
          HEAT1D_RUN(32)
        }
      }
      if constexpr (sizeof(F) == 4 && kLarge) {
        switch (m) {
          HEAT1D_RUN(40)
          HEAT1D_RUN(48)
          HEAT1D_RUN(56)
          HEAT1D_RUN(64)
        }
      }
      break;
  }
#undef HEAT1D_RUN
}

template <typename F>
__global__ __launch_bounds__(kBatchWaves * kWave) void batched_kernel(const BatchDev<F> b) {
  __shared__ F lds[8 * kBatchWaves];
  __shared__ int s_idx[kGroups + 1];
  __shared__ int s_count[kGroups];
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (threadIdx.x < kGroups) s_count[threadIdx.x] = 0;
  __syncthreads();

  const bool small_first = (int)blockIdx.x < b.small_first;
  // queues in the order 0, 1, 2, or 1, 2, 0 for the small-first workgroups;
  // each phase's code appears once
  for (int step = 0; step < 3; ++step) {
    const int q = small_first ? (step + 1) % 3 : step;
    if (q == 0) {
      // whole-workgroup rods (after the group phase, every wavefront is done
      // with the groups' LDS slots once all have arrived)
      if (step > 0) __syncthreads();
      for (;;) {
        if (threadIdx.x == 0) s_idx[kGroups] = atomicAdd(&b.heads[0], 1);
        __syncthreads();
        const int idx = s_idx[kGroups];
        __syncthreads();
        if (idx >= b.count[0]) break;
        run_one<F, RodSync::kWorkgroup>(b, b.order[0][idx], lds, kBatchWaves, wave, lane,
                                        nullptr, nullptr);
      }
    } else if (q == 1) {
      // rods on groups of kGroupWaves wavefronts
      const int g = wave / kGroupWaves;
      const int gw = wave % kGroupWaves;
      F* glds = lds + g * 8 * kGroupWaves;
      int epoch = 0;
      for (;;) {
        if (gw == 0 && lane == 0) s_idx[g] = atomicAdd(&b.heads[1], 1);
        group_barrier(&s_count[g], kGroupWaves, &epoch);
        const int idx = s_idx[g];
        group_barrier(&s_count[g], kGroupWaves, &epoch);
        if (idx >= b.count[1]) break;
        run_one<F, RodSync::kGroup>(b, b.order[1][idx], glds, kGroupWaves, gw, lane,
                                    &s_count[g], &epoch);
      }
    } else {
      // one rod per wavefront
      for (;;) {
        int idx = 0;
        if (lane == 0) idx = atomicAdd(&b.heads[2], 1);
        idx = __builtin_amdgcn_readlane(idx, 0);
        if (idx >= b.count[2]) break;
        run_one<F, RodSync::kWave>(b, b.order[2][idx], nullptr, 1, 0, lane, nullptr, nullptr);
      }
    }
  }
}

__global__ void fill_i32_kernel(int32_t* p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Points per lane: wavefront and group rods stay within 128 bytes per lane,
// where pinning the rod end is a direct register-indexed write; workgroup rods
// go up to the register budget of one wavefront in 16.
int batched_mmax(int dtype) { return dtype == 0 ? 64 : 32; }
int batched_mmax_small(int dtype) { return dtype == 0 ? 32 : 16; }
int batched_wave_capacity(int dtype) { return kWave * batched_mmax_small(dtype); }
int batched_group_capacity(int dtype) { return kGroupWaves * kWave * batched_mmax_small(dtype); }
int batched_wg_capacity(int dtype) { return kBatchWaves * kWave * batched_mmax(dtype); }

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0, s,
                     p, v, n);
  return hipGetLastError();
}

template <typename F>
static void batched_launch(const BatchedLaunch& a, hipStream_t s) {
  BatchDev<F> b;
  b.in = reinterpret_cast<const F*>(a.in);
  b.out = reinterpret_cast<F*>(a.out);
  b.offsets = a.offsets;
  b.r = a.r;
  b.c1 = a.c1;
  b.cN = a.cN;
  b.K = a.K;
  for (int i = 0; i < 3; ++i) {
    b.order[i] = a.order[i];
    b.count[i] = a.count[i];
  }
  b.heads = a.heads;
  b.small_first = a.small_first;
  hipLaunchKernelGGL(batched_kernel<F>, dim3((unsigned)a.groups), dim3(kBatchWaves * kWave), 0, s,
                     b);
}

hipError_t launch_batched(const BatchedLaunch& a, hipStream_t s) {
  hipError_t e = launch_fill_i32(a.heads, 0, 3, s);
  if (e != hipSuccess) return e;
  if (a.dtype == 0)
    batched_launch<float>(a, s);
  else
    batched_launch<double>(a, s);
  return hipGetLastError();
}

}  // namespace heat1d
