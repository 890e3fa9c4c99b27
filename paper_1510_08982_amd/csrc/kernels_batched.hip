// kernels_batched.hip -- thousands of independent rods of uneven length, step
// count and r in one persistent launch.
//
// One workgroup of 16 wavefronts runs per compute unit.  Phase 1: the whole
// workgroup takes rods from the "large" queue (longest N*K first) and runs each
// resident in registers, neighbouring wavefronts trading edge points through
// LDS behind one barrier per step.  Phase 2, once that queue is empty: every
// wavefront independently takes rods from the "small" queue and runs each in
// its own registers with DPP lane exchange only, no barrier at all.  Small rods
// thus fill the tail left by the large ones.  The points-per-lane count M of a
// rod is the smallest instantiated value that holds it.
#include "heat1d_device.h"
#include "heat1d_launch.h"
#include "heat1d_rod.h"

namespace heat1d {

constexpr int kBatchWaves = 16;

template <typename F>
struct BatchDev {
  const F* in;
  F* out;
  const int64_t* offsets;
  const double* r;
  const double* c1;
  const double* cN;
  const int32_t* K;
  const int32_t* order_wg;
  int32_t n_wg;
  const int32_t* order_wave;
  int32_t n_wave;
  int32_t* heads;
};

// Smallest supported M with capacity >= n for a block of `lanes` lanes.
__device__ __forceinline__ int pick_m(int n, int lanes) {
  const int need = (n + lanes - 1) / lanes;
  if (need <= 4) return 4;
  if (need <= 6) return 6;
  if (need <= 8) return 8;
  if (need <= 12) return 12;
  if (need <= 16) return 16;
  if (need <= 24) return 24;
  if (need <= 32) return 32;
  if (need <= 48) return 48;
  return 64;
}

template <typename F, bool kWG>
__device__ __forceinline__ void run_one(const BatchDev<F>& b, int rod, F* lds, int nwaves,
                                        int wave, int lane) {
  const int64_t off = b.offsets[rod];
  const int n = (int)(b.offsets[rod + 1] - off);
  const F r = (F)b.r[rod], c1 = (F)b.c1[rod], cN = (F)b.cN[rod];
  const int K = b.K[rod];
  const F* src = b.in + off;
  F* dst = b.out + off;
  const int m = uniform(pick_m(n, nwaves * kWave));
#define HEAT1D_RUN(MM)                                                                   \
  case MM:                                                                               \
    rod_resident<F, MM, kWG>(src, dst, n, K, r, c1, cN, lds, nwaves, wave, lane, false); \
    break;
  switch (m) {
    HEAT1D_RUN(4)
    HEAT1D_RUN(6)
    HEAT1D_RUN(8)
    HEAT1D_RUN(12)
    HEAT1D_RUN(16)
    HEAT1D_RUN(24)
    HEAT1D_RUN(32)
    default:
      if constexpr (sizeof(F) == 4) {
        switch (m) {
          HEAT1D_RUN(48)
          HEAT1D_RUN(64)
        }
      }
      break;
  }
#undef HEAT1D_RUN
}

template <typename F>
__global__ __launch_bounds__(kBatchWaves * kWave) void batched_kernel(const BatchDev<F> b) {
  __shared__ F lds[4 * kBatchWaves];
  __shared__ int s_idx;
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);

  // phase 1: whole-workgroup rods
  for (;;) {
    if (threadIdx.x == 0) s_idx = atomicAdd(&b.heads[0], 1);
    __syncthreads();
    const int idx = s_idx;
    __syncthreads();
    if (idx >= b.n_wg) break;
    run_one<F, true>(b, b.order_wg[idx], lds, kBatchWaves, wave, lane);
  }
  // phase 2: one rod per wavefront
  for (;;) {
    int idx = 0;
    if (lane == 0) idx = atomicAdd(&b.heads[1], 1);
    idx = __builtin_amdgcn_readlane(idx, 0);
    if (idx >= b.n_wave) break;
    run_one<F, false>(b, b.order_wave[idx], nullptr, 1, 0, lane);
  }
}

__global__ void fill_i32_kernel(int32_t* p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

int batched_wave_capacity(int dtype) { return kWave * (dtype == 0 ? 64 : 32); }
int batched_wg_capacity(int dtype) { return kBatchWaves * kWave * (dtype == 0 ? 64 : 32); }

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
  b.order_wg = a.order_wg;
  b.n_wg = a.n_wg;
  b.order_wave = a.order_wave;
  b.n_wave = a.n_wave;
  b.heads = a.heads;
  hipLaunchKernelGGL(batched_kernel<F>, dim3((unsigned)a.groups), dim3(kBatchWaves * kWave), 0, s,
                     b);
}

hipError_t launch_batched(const BatchedLaunch& a, hipStream_t s) {
  hipError_t e = launch_fill_i32(a.heads, 0, 2, s);
  if (e != hipSuccess) return e;
  if (a.dtype == 0)
    batched_launch<float>(a, s);
  else
    batched_launch<double>(a, s);
  return hipGetLastError();
}

}  // namespace heat1d
