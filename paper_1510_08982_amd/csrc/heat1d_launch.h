// heat1d_launch.h -- host-side launchers of the gfx950 kernels (internal).
// Each kernels_*.hip file defines its kernels and the launchers declared here;
// heat1d_api.cpp validates arguments, plans and calls them.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace heat1d {

// Points per lane a kernel template is instantiated for.
bool tiled_supports(int dtype, int M);
bool resident_supports(int dtype, int M);

// Geometry of the depth-T tiled pass: a wavefront tile holds L = 64*M points,
// of which the middle L - 2H are written; H >= steps per pass, rounded up to the
// vector width.
struct TileGeom {
  int M;
  int H;
  int L;
  int Wout;
  int64_t tiles_per_rod;
};
TileGeom tile_geometry(int dtype, int M, int T, int64_t N);

// ---- synchronous kernels -------------------------------------------------
// in/out hold nrods rods of N points; out receives u after `steps` steps.
hipError_t launch_sync_step(int dtype, const void* in, void* out, int64_t N, int64_t nrods,
                            double r, double c1, double cN, hipStream_t s);
hipError_t launch_sync_tiled(int dtype, const TileGeom& g, const void* in, void* out, int64_t N,
                             int64_t nrods, int steps, double r, double c1, double cN,
                             hipStream_t s);
hipError_t launch_sync_resident(int dtype, int M, int waves, const void* in, void* out, int64_t N,
                                int64_t nrods, int64_t K, double r, double c1, double cN,
                                hipStream_t s);
// Copy with the Dirichlet ends imposed (K = 0).
hipError_t launch_impose_ends(int dtype, const void* in, void* out, int64_t N, int64_t nrods,
                              double c1, double cN, hipStream_t s);

// ---- asynchronous persistent kernel --------------------------------------
struct AsyncLaunch {
  int dtype;
  int M;
  int waves;
  const void* in;
  void* out;
  int64_t N;
  int32_t P;
  int32_t K;
  int32_t d;
  int32_t Q;
  uint64_t seed;
  int32_t mode;
  double r, c1, cN;
  void* ring;      // [P][2][Q] tagged slots (uint64 words; 2 per slot for FP64)
  int32_t* prog;   // [P][2] newest-step hints
  int32_t* err;    // [0] status, [1] abort flag
  int64_t* stats;  // nullable, d+3 entries
  int64_t watchdog;
  int32_t remap;   // 1: keep neighbouring subdomains on one XCD
};
bool async_supports(int dtype, int M);
hipError_t launch_async_prepare(const AsyncLaunch& a, hipStream_t s);
hipError_t launch_async(const AsyncLaunch& a, hipStream_t s);
int async_max_resident_groups(int dtype, int M, int waves, int Q);
hipError_t launch_delay_schedule(int32_t P, int64_t K, int32_t d, uint64_t seed, uint8_t* out,
                                 hipStream_t s);

// ---- batched persistent kernel -------------------------------------------
struct BatchedLaunch {
  int dtype;
  const void* in;
  void* out;
  const int64_t* offsets;
  const double* r;
  const double* c1;
  const double* cN;
  const int32_t* K;
  const int32_t* order_wg;    // rods run by a whole workgroup, longest first
  int32_t n_wg;
  const int32_t* order_wave;  // rods run by a single wavefront, longest first
  int32_t n_wave;
  int32_t* heads;             // two queue counters
  int32_t groups;             // persistent workgroups
};
hipError_t launch_batched(const BatchedLaunch& b, hipStream_t s);
int batched_wave_capacity(int dtype);  // largest rod one wavefront holds
int batched_wg_capacity(int dtype);    // largest rod one workgroup holds
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);

// ---- adjoint -------------------------------------------------------------
// Record pass: from state `in` (time k0) advance `len-1` steps, writing the
// state after step i (i = 1..len-1) to states + (i-1)*stride elements.
hipError_t launch_record(int dtype, const TileGeom& g, const void* in, void* states,
                         int64_t stride, int64_t N, int64_t nrods, int len, double r, double c1,
                         double cN, hipStream_t s);
// Backward sweep over one stretch of `len` steps.  lam_in = lambda(k0+len),
// lam_out = lambda(k0); u(k0) is `u_first`, u(k0+i) for i >= 1 is
// states + (i-1)*stride.  partials[rod*tiles_per_rod + tile] receives the tile's
// dL/dr contribution (double).
hipError_t launch_adjoint_sweep(int dtype, const TileGeom& g, const void* lam_in, void* lam_out,
                                const void* u_first, const void* states, int64_t stride,
                                int64_t N, int64_t nrods, int len, double r, double* partials,
                                hipStream_t s);
// grad_r[b] = sum over segments s and tiles t of partials[s][b][t], in order.
hipError_t launch_reduce_partials(const double* partials, int64_t nseg, int64_t nrods,
                                  int64_t tiles_per_rod, double* grad_r, hipStream_t s);

}  // namespace heat1d
