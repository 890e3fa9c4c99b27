// kernels_observe.hip -- the l2 norm of a state, an observable of the run
// recorded every S steps off the hot loop (it stands in for the full history
// of states the paper keeps, Section 4).
#include <algorithm>

#include "heat1d_observe.h"

namespace heat1d {

constexpr int kNormThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kNormThreads / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  return sh[0];
}

// Block (c, b): sum of squares of points [c*chunk, (c+1)*chunk) of rod b,
// thread t taking points c*chunk + t, + 256, ... in order; with pin_ends the
// two end points count as c1 and cN.
template <typename F>
__global__ __launch_bounds__(kNormThreads) void norm_chunks_kernel(const F* __restrict__ u,
                                                                   int64_t N, double c1, double cN,
                                                                   int pin_ends,
                                                                   double* __restrict__ partials) {
  __shared__ double sh[kNormThreads];
  const int64_t c = blockIdx.x, b = blockIdx.y;
  const int64_t nch = gridDim.x;
  const F* __restrict__ rod = u + b * N;
  const int64_t i0 = c * kNormChunk;
  const int64_t i1 = i0 + kNormChunk < N ? i0 + kNormChunk : N;
  double acc = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kNormThreads) {
    const double v = (pin_ends && i == 0) ? c1 : ((pin_ends && i == N - 1) ? cN : (double)rod[i]);
    acc = fma(v, v, acc);
  }
  const double tot = block_sum(acc, sh);
  if (threadIdx.x == 0) partials[b * nch + c] = tot;
}

// out[b * out_stride] = sqrt(sum of the rod's chunk sums, in order).
__global__ __launch_bounds__(kNormThreads) void norm_finish_kernel(const double* __restrict__ partials,
                                                                   int64_t nch,
                                                                   double* __restrict__ out,
                                                                   int64_t out_stride) {
  __shared__ double sh[kNormThreads];
  const int64_t b = blockIdx.x;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < nch; i += kNormThreads) acc += partials[b * nch + i];
  const double tot = block_sum(acc, sh);
  if (threadIdx.x == 0) out[b * out_stride] = sqrt(tot);
}

hipError_t launch_state_norms(int dtype, const void* u, int64_t N, int64_t nrods, double c1,
                              double cN, double* partials, double* out, int64_t out_stride,
                              hipStream_t s, bool pin_ends) {
  if (N < 1 || nrods < 1 || nrods > 65535) return hipErrorInvalidValue;
  const int64_t nch = (N + kNormChunk - 1) / kNormChunk;
  const dim3 grid((unsigned)nch, (unsigned)nrods);
  if (dtype == 0)
    hipLaunchKernelGGL(norm_chunks_kernel<float>, grid, dim3(kNormThreads), 0, s,
                       (const float*)u, N, c1, cN, pin_ends ? 1 : 0, partials);
  else
    hipLaunchKernelGGL(norm_chunks_kernel<double>, grid, dim3(kNormThreads), 0, s,
                       (const double*)u, N, c1, cN, pin_ends ? 1 : 0, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(norm_finish_kernel, dim3((unsigned)nrods), dim3(kNormThreads), 0, s,
                     (const double*)partials, nch, out, out_stride);
  return hipGetLastError();
}

// Dot products of every rod b of g (nrods rods of N points) with w and with w
// read back to front, per chunk of kNormChunk points: partials[(b*nch + c)*2 + 0/1].
template <typename F>
__global__ __launch_bounds__(kNormThreads) void dot_chunks_kernel(const F* __restrict__ g,
                                                                  const F* __restrict__ w,
                                                                  int64_t N,
                                                                  double* __restrict__ partials) {
  __shared__ double sh[kNormThreads];
  const int64_t c = blockIdx.x, b = blockIdx.y;
  const int64_t nch = gridDim.x;
  const F* __restrict__ rod = g + b * N;
  const int64_t i0 = c * kNormChunk;
  const int64_t i1 = i0 + kNormChunk < N ? i0 + kNormChunk : N;
  double a0 = 0.0, a1 = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kNormThreads) {
    const double gi = (double)rod[i];
    a0 = fma(gi, (double)w[i], a0);
    a1 = fma(gi, (double)w[N - 1 - i], a1);
  }
  const double t0 = block_sum(a0, sh);
  __syncthreads();
  const double t1 = block_sum(a1, sh);
  if (threadIdx.x == 0) {
    partials[(b * nch + c) * 2] = t0;
    partials[(b * nch + c) * 2 + 1] = t1;
  }
}

// out0[b], out1[b] = the rod's chunk sums, in order.
__global__ __launch_bounds__(kNormThreads) void dot_finish_kernel(const double* __restrict__ partials,
                                                                  int64_t nch,
                                                                  double* __restrict__ out0,
                                                                  double* __restrict__ out1) {
  __shared__ double sh[kNormThreads];
  const int64_t b = blockIdx.x;
  double a0 = 0.0, a1 = 0.0;
  for (int64_t i = threadIdx.x; i < nch; i += kNormThreads) {
    a0 += partials[(b * nch + i) * 2];
    a1 += partials[(b * nch + i) * 2 + 1];
  }
  const double t0 = block_sum(a0, sh);
  __syncthreads();
  const double t1 = block_sum(a1, sh);
  if (threadIdx.x == 0) {
    out0[b] = t0;
    out1[b] = t1;
  }
}

hipError_t launch_mirror_dots(int dtype, const void* g, const void* w, int64_t N, int64_t nrods,
                              double* partials, double* out0, double* out1, hipStream_t s) {
  if (N < 1 || nrods < 1 || nrods > 65535) return hipErrorInvalidValue;
  const int64_t nch = (N + kNormChunk - 1) / kNormChunk;
  const dim3 grid((unsigned)nch, (unsigned)nrods);
  if (dtype == 0)
    hipLaunchKernelGGL(dot_chunks_kernel<float>, grid, dim3(kNormThreads), 0, s, (const float*)g,
                       (const float*)w, N, partials);
  else
    hipLaunchKernelGGL(dot_chunks_kernel<double>, grid, dim3(kNormThreads), 0, s, (const double*)g,
                       (const double*)w, N, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dot_finish_kernel, dim3((unsigned)nrods), dim3(kNormThreads), 0, s,
                     (const double*)partials, nch, out0, out1);
  return hipGetLastError();
}

__global__ void zero_words_kernel(uint32_t* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 4);
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t*)p, n);
  return hipGetLastError();
}

}  // namespace heat1d
