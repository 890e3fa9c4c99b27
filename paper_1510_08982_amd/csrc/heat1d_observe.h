// heat1d_observe.h -- launchers of the observable kernels (norms of a state).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace heat1d {

// Points per partial sum of the norm kernel, and the partials one state of
// nrods rods of N points needs.
constexpr int64_t kNormChunk = 8192;
inline int64_t norm_partials(int64_t N, int64_t nrods) {
  return nrods * ((N + kNormChunk - 1) / kNormChunk);
}

// out[b * out_stride] = ||u_b||_2 for each of the nrods rods of N points of the
// state u (FP32 or FP64), its ends read as c1 and cN (the state a step sees)
// when pin_ends, else as stored (a ring).  Squares are summed in double, per
// chunk of kNormChunk points and then per rod, each in a fixed order (the same
// bits on every run).  partials: norm_partials(N, nrods) doubles of scratch.
hipError_t launch_state_norms(int dtype, const void* u, int64_t N, int64_t nrods, double c1,
                              double cN, double* partials, double* out, int64_t out_stride,
                              hipStream_t s, bool pin_ends = true);

// out0[b] = <g_b, w>, out1[b] = <g_b, w reversed> for each of the nrods rods
// g_b of N points and one rod w of N points (FP32 or FP64), summed in double
// per chunk of kNormChunk points and then per rod, in a fixed order.
// partials: 2 * norm_partials(N, nrods) doubles of scratch.
hipError_t launch_mirror_dots(int dtype, const void* g, const void* w, int64_t N, int64_t nrods,
                              double* partials, double* out0, double* out1, hipStream_t s);

// Zero `bytes` (a multiple of 4) at p with a kernel (no memset node in a graph).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

}  // namespace heat1d
