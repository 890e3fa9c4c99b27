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
                            double r, double c1, double cN, hipStream_t s, bool ring = false);
// The periodic ring (Section 5.3): tile t writes ring points [t*Wout, (t+1)*Wout)
// and reads from t*Wout - H on, modulo N; ring_geometry counts those tiles.
TileGeom ring_geometry(int dtype, int M, int T, int64_t N);
hipError_t launch_sync_ring(int dtype, const TileGeom& g, const void* in, void* out, int64_t N,
                            int64_t nrods, int steps, double r, int fuse, hipStream_t s);
// fuse = S: steps per register sweep on tiles without a rod end (1, 2, 4);
// fused_supports() lists the instantiated (M, S) pairs.
bool fused_supports(int dtype, int M, int S);
hipError_t launch_sync_tiled(int dtype, const TileGeom& g, const void* in, void* out, int64_t N,
                             int64_t nrods, int steps, double r, double c1, double cN, int fuse,
                             hipStream_t s);
// Wide tiles: one tile of G*64*M points per workgroup of G wavefronts, the
// wavefront boundaries traded through LDS once per sweep.  g is the geometry
// of the whole tile (tile_geometry with G*M points per lane); results are bit
// for bit those of the tiled kernel for S = 1 (fused sweeps round alike too).
bool wide_supports(int dtype, int M, int S, int G);
hipError_t launch_sync_wide(int dtype, const TileGeom& g, int M, int G, const void* in, void* out,
                            int64_t N, int64_t nrods, int steps, double r, double c1, double cN,
                            int fuse, hipStream_t s);
// The ring in wide tiles: g = ring_geometry with G*M points per lane; the
// (M, S, G) of wide_supports.  Bit for bit the narrow ring's results.
hipError_t launch_sync_wide_ring(int dtype, const TileGeom& g, int M, int G, const void* in,
                                 void* out, int64_t N, int64_t nrods, int steps, double r,
                                 int fuse, hipStream_t s);

// Persistent pipelined form of the tiled pass (same results, bit for bit): a
// grid of resident wavefronts that prefetch their next tile while computing.
// It moves whole 16-byte vectors only (in/out 16-byte aligned, N a multiple of
// the vector width: 4 FP32 / 2 FP64 elements) and needs N > one tile.
bool pipelined_applies(int dtype, const TileGeom& g, const void* in, const void* out, int64_t N);
hipError_t launch_sync_pipelined(int dtype, const TileGeom& g, const void* in, void* out,
                                 int64_t N, int64_t nrods, int steps, double r, double c1,
                                 double cN, int fuse, hipStream_t s);
// Instantiated (M, S) pairs: every M with S = 1, a subset with S = 2 and 4.
#define HEAT1D_FOR_EACH_F32(X)                                                    \
  X(float, 4, 1) X(float, 8, 1) X(float, 16, 1) X(float, 24, 1) X(float, 32, 1)  \
  X(float, 40, 1) X(float, 48, 1) X(float, 64, 1)                                \
  X(float, 16, 2) X(float, 32, 2) X(float, 48, 2) X(float, 64, 2)                \
  X(float, 16, 4) X(float, 32, 4) X(float, 48, 4) X(float, 64, 4)
#define HEAT1D_FOR_EACH_F64(X)                                                    \
  X(double, 2, 1) X(double, 4, 1) X(double, 8, 1) X(double, 12, 1)               \
  X(double, 16, 1) X(double, 20, 1) X(double, 24, 1) X(double, 32, 1)            \
  X(double, 8, 2) X(double, 16, 2) X(double, 24, 2) X(double, 32, 2)             \
  X(double, 8, 4) X(double, 16, 4) X(double, 24, 4) X(double, 32, 4)


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
  int32_t jitter;  // seeded pause per step: 0..jitter short sleeps (0 = none)
  int32_t periodic;  // 1: ring of Section 5.3, subdomains 0 and P-1 neighbours (P >= 2)
  int32_t sched;     // emulated mode: delay schedule (sched_delay in heat1d_delays.h)
};
bool async_supports(int dtype, int M);
hipError_t launch_async_prepare(const AsyncLaunch& a, hipStream_t s);
hipError_t launch_async(const AsyncLaunch& a, hipStream_t s);
int async_max_resident_groups(int dtype, int M, int waves, int Q);
hipError_t launch_delay_schedule(int32_t P, int64_t K, int32_t d, uint64_t seed, uint8_t* out,
                                 hipStream_t s);
// Allocation-free run: the per-device address of the library's fixed scratch
// array of kNoAllocScratchBytes (looked up once per device), and a one-thread
// copy of the run's status word to a caller's device int32.
constexpr size_t kNoAllocScratchBytes = (size_t)4 << 20;
hipError_t async_noalloc_scratch(void** ptr);
hipError_t launch_copy_status(const int32_t* err, int32_t* status, hipStream_t s);

// ---- gradients through the emulated asynchronous iteration ---------------
// Lockstep replay of Eq.4 in the emulated mode (one launch per step) and its
// transpose.  E and LE: (K+1) x P x 2 edge records of u and lambda (element
// type of the state): [k][b][0] the point lo(b)-1, [k][b][1] the point lo(b),
// for the edges b = 1..P-1 (on the ring also edge 0, between point N-1 and
// point 0).  lo: the partition table lo[0..P].  part: one double per
// workgroup of a step launch (async_adjoint_blocks), ends: two.
struct AsyncAdjStep {
  int dtype;
  int ring;   // 1: periodic ring of Section 5.3 (P >= 2), every point updated
  int sched;  // delay schedule (sched_delay in heat1d_delays.h)
  int64_t N;
  int P, K, d;
  uint64_t seed;
  double r, c1, cN;
  void* E;
  void* LE;
  const int64_t* lo;
  double* part;
  double* ends;
  // tile orders of the tiled lockstep and transpose launches (async_tiled_order)
  const int* ord_lock;
  const int* ord_adj;
};
int64_t async_adjoint_blocks(int64_t N);
hipError_t launch_async_partition(int64_t* lo, int64_t N, int P, hipStream_t s);
hipError_t launch_async_edges(int dtype, const void* u, void* Ek, const int64_t* lo, int P,
                              int64_t N, int ring, hipStream_t s);
// u(k+1) = step k of Eq.4 from u(k) = cur; record != 0 also writes E[k+1].
hipError_t launch_async_lockstep(const AsyncAdjStep& a, const void* cur, void* nxt, int k,
                                 int record, hipStream_t s);
// The same steps on register tiles, at most async_tiled_depth() per launch,
// for rods (or rings, P >= 2) whose subdomains are longer than one tile (bit
// for bit the per-step launches): from the state `in` of step k0, `steps` steps; when
// states is not NULL, every state u(k) with k - kc a positive multiple of
// async_tiled_store_every() goes to states + ((k-kc)/every - 1)*stride; the
// last state to `out` unless it is NULL.
bool async_tiled_applies(int64_t N, int P, int d);
int async_tiled_depth();
int async_tiled_store_every();
hipError_t launch_async_lockstep_tiled(const AsyncAdjStep& a, const void* in, void* out,
                                       void* states, int64_t stride, int kc, int k0, int steps,
                                       int record, hipStream_t s);
// The transpose steps k0+steps-1 .. k0 on register tiles, lambda in registers;
// u from the sparse states of the replay (u_first for k == kc, st_base +
// ((k-kc)/every - 1)*stride for the other multiples of every above kc) and
// recomputed between them; k0 - kc a multiple of every; lambda bit for bit
// that of the per-step kernel; dL/dr summed per tile into part[t]
// (async_tiled_tiles slots), dL/dc1 and dL/dcN into ends.
int64_t async_tiled_tiles(int dtype, int64_t N);
// The order in which the tiled launches take their tiles: those holding a
// subdomain edge (the longest-running) first, then the rest, each in tile
// order.  ord_lock and ord_adj hold async_tiled_tiles(dtype, N) ints each.
hipError_t launch_async_tiled_order(const AsyncAdjStep& a, int* ord_lock, int* ord_adj,
                                    hipStream_t s);
hipError_t launch_async_adjoint_tiled(const AsyncAdjStep& a, const void* lam_in, void* lam_out,
                                      const void* u_first, const void* st_base, int64_t stride,
                                      int kc, int k0, int steps, hipStream_t s);
// lambda(k) from lambda(k+1) and u(k), LE[k] and the step's dL/dr, dL/dc1,
// dL/dcN terms (added to part and ends).
hipError_t launch_async_adjoint_step(const AsyncAdjStep& a, const void* lam1, void* lam0,
                                     const void* u, int k, hipStream_t s);
hipError_t launch_async_adjoint_ends(int dtype, const void* gK, int64_t N, const double* ends,
                                     double* grad_c1, double* grad_cN, int ring, hipStream_t s);
hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t s);

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
  const int32_t* order[3];  // rods run by the workgroup / a 4-wavefront group /
                            // one wavefront, each longest first
  int32_t count[3];
  int32_t* heads;           // three queue counters
  int32_t groups;           // persistent workgroups
  int32_t small_first;      // of which these start with the group and wavefront queues
};
hipError_t launch_batched(const BatchedLaunch& b, hipStream_t s);
int batched_wave_capacity(int dtype);   // largest rod one wavefront holds
int batched_group_capacity(int dtype);  // largest rod a 4-wavefront group holds
int batched_wg_capacity(int dtype);     // largest rod one workgroup holds
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);

// ---- adjoint -------------------------------------------------------------
// One register-resident sub-stretch of the backward sweep: from u(k0) (the
// sub-stretch's first state) recompute the Laplacians of u(k0..k0+len-1) in
// registers, then lambda(k0+len) -> lambda(k0), writing the dL/dr sum of tile
// t of rod b to partials[b*part_stride + part_off + t].
// len <= stretch_steps(dtype).
struct StretchArgs {
  const void* u_start;
  const void* lam_in;
  void* lam_out;
  int64_t N;
  int64_t nrods;
  int len;
  double r, c1, cN;
  double* partials;
  int64_t part_stride;
  int64_t part_off;
};
int stretch_steps(int dtype);
TileGeom stretch_geometry(int dtype, int64_t N);
hipError_t launch_adjoint_stretch(int dtype, const TileGeom& g, const StretchArgs& a,
                                  hipStream_t s);
// grad_r[b] = sum of partials[b*n .. b*n + n), in a fixed order (the
// partials are scratch: long rows are reduced in place).
hipError_t launch_reduce_partials(double* partials, int64_t n, int64_t nrods, double* grad_r,
                                  hipStream_t s);

}  // namespace heat1d
