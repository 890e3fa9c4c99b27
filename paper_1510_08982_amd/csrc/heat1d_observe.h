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
// state u (FP32 or FP64), its ends read as c1 and cN (the state a step sees).
// Squares are summed in double, per chunk of kNormChunk points and then per
// rod, each in a fixed order (the same bits on every run).  partials:
// norm_partials(N, nrods) doubles of scratch.
hipError_t launch_state_norms(int dtype, const void* u, int64_t N, int64_t nrods, double c1,
                              double cN, double* partials, double* out, int64_t out_stride,
                              hipStream_t s);

}  // namespace heat1d
