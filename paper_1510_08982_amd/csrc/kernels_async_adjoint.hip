// kernels_async_adjoint.hip -- gradients through the emulated asynchronous
// iteration (Eq.4 of Section 3) of one rod of any length, with checkpoints
// every S ~ sqrt(K) steps.
//
// In the emulated mode the delays are a fixed function of (seed, k, p, side),
// so the iteration is a fixed linear map of u(0) and the ends, and neither its
// forward replay nor its transpose needs any real concurrency: both run in
// lockstep, one launch per step over the whole rod, one thread per point.  A
// delayed read only ever reaches one of the two points next to a subdomain
// edge, so instead of the last d+1 whole states the run keeps a record of
// those points alone: E[k][b] = (u_{lo(b)-1}(k), u_{lo(b)}(k)) for every step k
// and every edge b = 1..P-1 (lo(b) = floor(b N / P), the partition of
// Section 2), 2 (K+1) P values.  The backward sweep keeps the same record of
// lambda (LE), from which an edge point gathers the contributions of every
// later step whose delayed read landed on its value: the neighbour across
// edge b read u_j(k) at the steps k' in k..k+d with max(k' - delta(k'), 0) = k,
// so lambda_j(k) collects r lambda_{j+-1}(k'+1) over exactly those k'.
//
// On the periodic ring of Section 5.3 (P >= 2) every point is updated and
// edge 0 is the wrap between subdomain P-1 and subdomain 0: E[k][0] =
// (u_{N-1}(k), u_0(k)), and subdomain p's right edge is edge (p+1) mod P.
//
// Steps are HBM-bound: a forward step reads and writes the state (2 s bytes
// per point), a backward step reads lambda(k+1) and u(k) and writes lambda(k)
// (3 s bytes per point); the edge records add 2 values per edge and step.
#include <algorithm>

#include "heat1d_delays.h"
#include "heat1d_device.h"
#include "heat1d_launch.h"

namespace heat1d {

namespace {

constexpr int kThreads = 256;

// Subdomain of point i from the partition table lo[0..P] (lo[P] = N): an
// estimate from i P / N, then corrected against the table (at most a step or
// two either way).
__device__ __forceinline__ int sub_of(int64_t i, const int64_t* __restrict__ lo, int P,
                                      double pscale) {
  int p = (int)((double)i * pscale);
  p = p < 0 ? 0 : (p > P - 1 ? P - 1 : p);
  while (p > 0 && lo[p] > i) --p;
  while (p + 1 < P && lo[p + 1] <= i) ++p;
  return p;
}

// The same subdomain from the partition's formula lo(p) = floor(p N / P)
// (what partition_kernel writes), with no table reads: a tile finds its edge
// before its first load returns.
__device__ __forceinline__ int64_t part_lo(int64_t p, int64_t N, int P) { return p * N / P; }

__device__ __forceinline__ int sub_of_formula(int64_t i, int64_t N, int P, double pscale) {
  int p = (int)((double)i * pscale);
  p = p < 0 ? 0 : (p > P - 1 ? P - 1 : p);
  while (p > 0 && part_lo(p, N, P) > i) --p;
  while (p + 1 < P && part_lo(p + 1, N, P) <= i) ++p;
  return p;
}

__global__ void partition_kernel(int64_t* __restrict__ lo, int64_t N, int P) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p <= P) lo[p] = (int64_t)p * N / P;
}

// E[k][b] for every edge b from the state u(k) (edge 0 on the ring only).
template <typename F>
__global__ void edges_from_state_kernel(const F* __restrict__ u, F* __restrict__ Ek,
                                        const int64_t* __restrict__ lo, int P, int64_t N,
                                        int ring) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= P || (b == 0 && !ring)) return;
  Ek[2 * b] = u[b == 0 ? N - 1 : lo[b] - 1];
  Ek[2 * b + 1] = u[lo[b]];
}

// Each thread takes kPts consecutive points (whole 16-byte vectors when the
// buffers allow), so that a wavefront keeps enough bytes in flight to stream
// at HBM rate; the two neighbours outside the group are read singly (they
// are in cache: the neighbouring threads load them).  The subdomain of the
// group's first point comes from the partition table; a group rarely holds
// an edge, and then only the points next to it take the delayed reads.
constexpr int kPts = 8;

// Edge flags of point i in subdomain p (p advanced past any edge before i).
// On the ring (P >= 2) subdomain 0 has a left edge and subdomain P-1 a right
// one; on the Dirichlet rod they end at the fixed points instead.
template <bool kRing>
struct EdgeScan {
  int p;
  int64_t lo_p, lo_p1;  // lo[p], lo[p+1]
  __device__ __forceinline__ void to(int64_t i, const int64_t* __restrict__ lo, int P) {
    while (p + 1 < P && lo_p1 <= i) {
      ++p;
      lo_p = lo_p1;
      lo_p1 = lo[p + 1];
    }
  }
  __device__ __forceinline__ bool first(int64_t i) const { return (kRing || p > 0) && i == lo_p; }
  __device__ __forceinline__ bool last(int64_t i, int P) const {
    return (kRing || p + 1 < P) && i == lo_p1 - 1;
  }
  // whether the group [i0, i0+n) holds no edge point (p is i0's subdomain)
  __device__ __forceinline__ bool none_in(int64_t i0, int n, int P) const {
    return !((kRing || p + 1 < P) && lo_p1 - 1 <= i0 + n - 1) && !((kRing || p > 0) && lo_p == i0);
  }
  // edge indices of the subdomain's left and right edges
  __device__ __forceinline__ int left_edge() const { return p; }
  __device__ __forceinline__ int right_edge(int P) const { return p + 1 == P ? 0 : p + 1; }
};

template <bool kRing>
__device__ __forceinline__ EdgeScan<kRing> edge_scan(int64_t i0, const int64_t* __restrict__ lo,
                                                     int P, double pscale) {
  EdgeScan<kRing> e;
  e.p = sub_of(i0, lo, P, pscale);
  e.lo_p = lo[e.p];
  e.lo_p1 = lo[e.p + 1];
  return e;
}

// u(k+1) from u(k): Eq.4 with the emulated delays, the ends held at c1, cN.
// A subdomain's first point reads its left neighbour, and its last point its
// right neighbour, at step max(k - delta, 0) from the edge record; every other
// read is of step k.  The points next to an edge also record their new value
// in E[k+1] (when record != 0; a replay leaves the record as the forward pass
// wrote it, which is the same values).
template <typename F, bool kRing>
__global__ __launch_bounds__(kThreads) void async_lockstep_kernel(
    const F* __restrict__ cur, F* __restrict__ nxt, F* __restrict__ E,
    const int64_t* __restrict__ lo, int64_t N, int P, int k, int d, uint64_t seed, int sched,
    F r, F c1, F cN, double pscale, int record, int aligned) {
  const int64_t i0 = ((int64_t)blockIdx.x * kThreads + threadIdx.x) * kPts;
  if (i0 >= N) return;
  F c[kPts], v[kPts];
  load_points<F, kPts>(c, cur, i0, N, aligned != 0);
  // (on the ring points 0 and N-1 are edge points: their wrapped reads come
  // from the edge record, never from these two)
  const F before = i0 >= 1 ? cur[i0 - 1] : F(0);
  const F after = i0 + kPts < N ? cur[i0 + kPts] : F(0);
  EdgeScan<kRing> es = edge_scan<kRing>(i0, lo, P, pscale);
  const bool plain = es.none_in(i0, kPts, P) && i0 >= 1 && i0 + kPts <= N - 1;
  if (plain) {
    // no end and no edge among the group's points: Eq.3 on all of them
#pragma unroll
    for (int j = 0; j < kPts; ++j)
      v[j] = eq3_step(j > 0 ? c[j - 1] : before, c[j], j + 1 < kPts ? c[j + 1] : after, r);
  } else {
#pragma unroll
    for (int j = 0; j < kPts; ++j) {
      const int64_t i = i0 + j;
      if (i >= N) { v[j] = F(0); continue; }
      es.to(i, lo, P);
      const bool first = es.first(i), last = es.last(i, P);
      F val;
      if (!kRing && i == 0) {
        val = c1;
      } else if (!kRing && i == N - 1) {
        val = cN;
      } else {
        F left = j > 0 ? c[j - 1] : before, right = j + 1 < kPts ? c[j + 1] : after;
        if (first) {
          const int dl = sched_delay(sched, seed, k, es.p, 0, P, d);
          left = E[((int64_t)(k - dl > 0 ? k - dl : 0) * P + es.left_edge()) * 2];
        }
        if (last) {
          const int dr = sched_delay(sched, seed, k, es.p, 1, P, d);
          right = E[((int64_t)(k - dr > 0 ? k - dr : 0) * P + es.right_edge(P)) * 2 + 1];
        }
        val = eq3_step(left, c[j], right, r);
      }
      v[j] = val;
      if (record) {
        if (first) E[((int64_t)(k + 1) * P + es.left_edge()) * 2 + 1] = val;
        if (last) E[((int64_t)(k + 1) * P + es.right_edge(P)) * 2] = val;
      }
    }
  }
  store_points<F, kPts>(v, nxt, i0, 0, 0, (int)(N - i0 < kPts ? N - i0 : kPts), aligned != 0);
}

// The same steps, `steps` <= H of them per launch, on register tiles (one
// wavefront per tile of L = 64 M points held in registers, neighbours by DPP,
// the middle L - 2H points stored; the tiles of TileSetup), for rods or rings
// whose subdomains are longer than a tile: then a tile holds at most one edge
// b, its two points a = lo(b)-1 and lo(b) at tile-local positions qa and qa+1.  Every point takes the plain step; the two edge points are then
// recomputed with their delayed reads, from a history of their last d+2
// values kept in LDS (filled from the edge record E for the steps before the
// launch, by the tile itself after).  A tile whose output range holds an edge
// point records its values in E (record != 0).  With `states` not NULL every
// state u(k) the launch computes with k - kc a positive multiple of kStoreEvery
// is stored at states + ((k - kc) / kStoreEvery - 1) * stride (the sparse
// replay of a stretch that starts at step kc); the last state goes to `out`
// unless it is NULL.
constexpr int kTileM = 16;
constexpr int kTileT = 32;
constexpr int kHistQ = 258;  // d + 2 slots for d <= 255
// The replay of a stretch stores every kStoreEvery-th state; the transpose
// recomputes the kStoreEvery-1 states between them in registers, so its tiles
// carry kStoreEvery-1 more halo points (kAdjT).
constexpr int kStoreEvery = 4;
constexpr int kAdjT = kTileT + kStoreEvery;
// Tiles per workgroup of the lockstep and transpose kernels.  A workgroup's
// tiles finish at different times (the one holding a subdomain edge runs
// longest), and its wavefront slots are refilled only once all of them are
// done, so one tile per workgroup keeps the CU's slots busy.
constexpr int kAdjWaves = 1;
static_assert(kTileT % kStoreEvery == 0, "launches start on kept states");

// Where a tile sits and what it holds.  Dirichlet rods: the tiles of the
// synchronous tiled pass (tile t from point t*Wout, the rod ends pinned by the
// tiles that hold them).  Rings: the ring tiles (tile t from ring index
// t*Wout - H, taken modulo N, output [H, H + min(Wout, N - t*Wout))), no
// pinned point.  The edge, if the tile holds one: edge b (0 on the ring is
// the wrap between point N-1 and point 0) with its point a = lo(b)-1 of
// subdomain pa at local qa and its point lo(b) at qa+1.
struct TileSetup {
  int64_t base;
  int lo_t, hi_t;
  bool left_end, right_end;
  int qN;
  bool has_edge;
  int b, pa, qa;
};

template <bool kRing>
__device__ __forceinline__ TileSetup tile_setup(int64_t t, int64_t tiles, int L, int H, int64_t N,
                                                int P, double pscale) {
  TileSetup s;
  const int Wout = L - 2 * H;
  if (kRing) {
    s.base = t * Wout - H;
    const int64_t rem = N - t * Wout;
    s.lo_t = H;
    s.hi_t = H + (rem < Wout ? (int)rem : Wout);
    s.left_end = s.right_end = false;
    s.qN = 0;
  } else {
    s.base = t * Wout;
    s.left_end = t == 0;
    const int64_t qN64 = N - 1 - s.base;
    s.right_end = qN64 < L;
    s.lo_t = s.left_end ? 0 : H;
    s.hi_t = (t == tiles - 1) ? (int)(N - s.base) : (L - H);
    s.qN = s.right_end ? (int)qN64 : 0;
  }
  s.has_edge = false;
  s.b = s.pa = s.qa = 0;
  if (P > 1) {
    int64_t g0 = s.base;
    if (kRing) {
      g0 = s.base % N;
      if (g0 < 0) g0 += N;
    }
    const int p0 = sub_of_formula(g0, N, P, pscale);
    if (kRing || p0 + 1 < P) {
      const int64_t lob = part_lo(p0 + 1, N, P);  // N for the last subdomain: the wrap edge
      if (lob <= g0 + L) {
        s.has_edge = true;
        s.b = p0 + 1 == P ? 0 : p0 + 1;
        s.pa = p0;
        s.qa = (int)(lob - 1 - g0);
      }
    }
  }
  s.b = uniform(s.b);
  s.pa = uniform(s.pa);
  s.qa = uniform(s.qa);
  return s;
}

// The lane's M points of a tile from local point 0 at index `base`: whole
// vectors inside the rod, taken modulo N on a ring tile that crosses the seam.
template <typename F, int M, bool kRing>
__device__ __forceinline__ void load_tile(F (&u)[M], const F* __restrict__ src, int64_t base,
                                          int q0, int L, int64_t N, bool aligned) {
  if (!kRing || (base >= 0 && base + L <= N)) {
    load_points<F, M>(u, src, base + q0, N, aligned);
  } else {
    int64_t g = (base + q0) % N;
    if (g < 0) g += N;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      u[j] = src[g];
      g = g + 1 == N ? 0 : g + 1;
    }
  }
}

// order[0..tiles): the tiles holding an edge, then the others, each in tile
// order (one workgroup; a chunk of 256 tiles per pass, places from ballots).
template <bool kRing>
__global__ __launch_bounds__(256) void tile_order_kernel(int* __restrict__ order, int64_t tiles,
                                                          int L, int H, int64_t N, int P,
                                                          double pscale) {
  __shared__ int cnt[2][4];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const uint64_t below = (1ull << lane) - 1;
  int64_t ne = 0;  // edge tiles in all
  for (int64_t c = 0; c < tiles; c += 256) {
    const int64_t t = c + threadIdx.x;
    const bool e = t < tiles && tile_setup<kRing>(t, tiles, L, H, N, P, pscale).has_edge;
    ne += __popcll(__ballot(e));
  }
  __syncthreads();
  if (lane == 0) cnt[0][w] = (int)ne;
  __syncthreads();
  int64_t pe = 0, pn = cnt[0][0] + cnt[0][1] + cnt[0][2] + cnt[0][3];
  for (int64_t c = 0; c < tiles; c += 256) {
    const int64_t t = c + threadIdx.x;
    const bool in = t < tiles;
    const bool e = in && tile_setup<kRing>(t, tiles, L, H, N, P, pscale).has_edge;
    const uint64_t me = __ballot(e), mn = __ballot(in && !e);
    __syncthreads();
    if (lane == 0) {
      cnt[0][w] = __popcll(me);
      cnt[1][w] = __popcll(mn);
    }
    __syncthreads();
    int be = 0, bn = 0;
    for (int i = 0; i < w; ++i) {
      be += cnt[0][i];
      bn += cnt[1][i];
    }
    if (e) order[pe + be + __popcll(me & below)] = (int)t;
    else if (in) order[pn + bn + __popcll(mn & below)] = (int)t;
    pe += cnt[0][0] + cnt[0][1] + cnt[0][2] + cnt[0][3];
    pn += cnt[1][0] + cnt[1][1] + cnt[1][2] + cnt[1][3];
  }
}

template <typename F, bool kRing>
__global__ __launch_bounds__(kAdjWaves * kWave) void async_lockstep_tiled_kernel(
    const F* __restrict__ in, F* __restrict__ out, F* __restrict__ states, int64_t stride,
    int kc, F* __restrict__ E, const int* __restrict__ order, int64_t N, int P, int k0,
    int steps, int d,
    uint64_t seed, int sched, F r, F c1, F cN, int64_t tiles, int H, double pscale, int record,
    int aligned) {
  constexpr int M = kTileM;
  constexpr int L = kWave * M;
  __shared__ F hist[kAdjWaves][2][kHistQ];
  __shared__ int pull[kAdjWaves][2][kTileT];  // max(k - dL, 0), max(k - dR, 0)
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int64_t v = (int64_t)blockIdx.x * kAdjWaves + w;
  if (v >= tiles) return;
  const int64_t t = order[v];
  // the tile's first point (as tile_setup places it), so the loads go out first
  const int64_t base = kRing ? t * (L - 2 * H) - H : t * (L - 2 * H);
  const int q0 = lane * M;
  const bool st_aligned = aligned != 0 && base >= 0;
  F u[M];
  load_tile<F, M, kRing>(u, in, base, q0, L, N, aligned != 0);
  const TileSetup ts = tile_setup<kRing>(t, tiles, L, H, N, P, pscale);
  const bool left_end = ts.left_end, right_end = ts.right_end;
  const int lo_t = ts.lo_t, hi_t = ts.hi_t;
  const int qN = ts.qN;
  const int lN = qN / M, jN = uniform(qN % M);
  // the edge in this tile, if any (wave-uniform)
  const bool has_edge = ts.has_edge;
  // a tile holding an edge has the longest chain of the launch: its wavefront
  // issues ahead of the plain tiles sharing its SIMD
  if (has_edge) __builtin_amdgcn_s_setprio(2);
  const int b = ts.b, pa = ts.pa, qa = ts.qa;
  const int qb = qa + 1;
  const int Q = d + 2;
  F* ha = hist[w][0];
  F* hb = hist[w][1];
  int* pL = pull[w][0];
  int* pR = pull[w][1];
  if (has_edge) {
    for (int j = lane; j < steps; j += kWave) {
      const int k = k0 + j;
      const int dL = sched_delay(sched, seed, k, b, 0, P, d);
      const int dR = sched_delay(sched, seed, k, pa, 1, P, d);
      pL[j] = k - dL > 0 ? k - dL : 0;
      pR[j] = k - dR > 0 ? k - dR : 0;
    }
    const int s0 = k0 - d > 0 ? k0 - d : 0;
    for (int s = s0 + lane; s <= k0; s += kWave) {
      ha[s % Q] = E[((int64_t)s * P + b) * 2];
      hb[s % Q] = E[((int64_t)s * P + b) * 2 + 1];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  const bool own_a = qa >= lo_t && qa < hi_t, own_b = qb >= lo_t && qb < hi_t;
  if (left_end) u[0] = (lane == 0) ? c1 : u[0];
  if (right_end) set_point<F, M>(u, jN, lane == lN, cN);
  for (int s = 0; s < steps; ++s) {
    const int k = k0 + s;
    F ua = F(0), ual = F(0), ub = F(0), ubr = F(0);
    if (has_edge) {
      ua = read_lane(get_point<F, M>(u, qa % M), qa / M);
      if (qa >= 1) ual = read_lane(get_point<F, M>(u, (qa - 1) % M), (qa - 1) / M);
      if (qb < L) ub = read_lane(get_point<F, M>(u, qb % M), qb / M);
      if (qb + 1 < L) ubr = read_lane(get_point<F, M>(u, (qb + 1) % M), (qb + 1) / M);
    }
    const F left = from_lower_lane(u[M - 1]);
    const F right = from_upper_lane(u[0]);
    lane_step<F, M>(u, left, right, r);
    if (has_edge) {
      const int ksR = pR[s], ksL = pL[s];
      const F rb = ksR == k ? ub : hb[ksR % Q];
      const F la = ksL == k ? ua : ha[ksL % Q];
      const F na = eq3_step(ual, ua, rb, r);
      const F nb = eq3_step(la, ub, ubr, r);
      set_point<F, M>(u, qa % M, lane == qa / M, na);
      if (qb < L) set_point<F, M>(u, qb % M, lane == qb / M, nb);
      if (lane == 0) {
        ha[(k + 1) % Q] = na;
        hb[(k + 1) % Q] = nb;
        if (record && own_a) E[((int64_t)(k + 1) * P + b) * 2] = na;
        if (record && own_b) E[((int64_t)(k + 1) * P + b) * 2 + 1] = nb;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (left_end) u[0] = (lane == 0) ? c1 : u[0];
    if (right_end) set_point<F, M>(u, jN, lane == lN, cN);
    if (states && (k + 1 - kc) % kStoreEvery == 0)
      store_points<F, M>(u, states + (int64_t)((k + 1 - kc) / kStoreEvery - 1) * stride,
                         base + q0, q0, lo_t, hi_t, st_aligned);
  }
  if (out) store_points<F, M>(u, out, base + q0, q0, lo_t, hi_t, st_aligned);
}

// The transpose steps k0+steps-1 down to k0 on register tiles: lambda of the
// tile's points stays in registers across the launch's steps.  The states come
// from the sparse replay: u(k) is stored for k - kc a multiple of kStoreEvery
// (u_first for k == kc, the stretch's checkpoint; st_base + ((k-kc)/kStoreEvery - 1)
// * stride above it), and the up to kStoreEvery-1 states above each stored one
// are recomputed in registers (Eq.4 with the delayed edge reads taken from the
// edge record E) before the transpose steps that use them; the next stored
// state is loaded while the current group is computed.  k0 - kc is a multiple
// of kStoreEvery.  Every point takes the plain transpose step (lambda_i(k)
// from lambda_{i+-1}(k+1), neighbours by DPP); the two edge points are then
// recomputed with the contributions gathered from the later steps whose
// delayed reads landed on them, from an LDS history of their lambda (filled
// from LE for the steps above the launch), in the order of the per-step
// kernel, so lambda is bit for bit the same.  dL/dr over the tile's own
// output points (the edge points' delayed Laplacians as a correction of the
// plain ones), each step's terms of a lane summed in the state precision and
// those sums in double, into part[t]; dL/dc1 and dL/dcN by the tiles that own
// points 1 and N-2.  The tiles carry kStoreEvery-1 halo points more
// than the steps need (the recomputed states lose one valid point per step at
// each tile end).
template <typename F, bool kRing>
__global__ __launch_bounds__(kAdjWaves * kWave) void async_adjoint_tiled_kernel(
    const F* __restrict__ lam_in, F* __restrict__ lam_out, const F* __restrict__ u_first,
    const F* __restrict__ st_base, int64_t stride, int kc, const F* __restrict__ E,
    F* __restrict__ LE, const int* __restrict__ order, int64_t N, int P, int k0, int steps,
    int K, int d, uint64_t seed, int sched, F r, F c1, F cN, int64_t tiles, int H, double pscale,
    double* __restrict__ part, double* __restrict__ ends, int aligned) {
  constexpr int M = kTileM;
  constexpr int L = kWave * M;
  constexpr int G = kStoreEvery;
  __shared__ F hist[kAdjWaves][2][kHistQ];
  // per edge tile, for the launch's steps: the delayed edge values its steps
  // read, and the step whose read each later step's delay lands on
  __shared__ F edly[kAdjWaves][2][kTileT];
  __shared__ int pull[kAdjWaves][2][kTileT + kHistQ];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int64_t v = (int64_t)blockIdx.x * kAdjWaves + w;
  if (v >= tiles) return;
  const int64_t t = order[v];
  const int64_t base = kRing ? t * (L - 2 * H) - H : t * (L - 2 * H);
  const int q0 = lane * M;
  F l[M];
  load_tile<F, M, kRing>(l, lam_in, base, q0, L, N, aligned != 0);
  const TileSetup ts = tile_setup<kRing>(t, tiles, L, H, N, P, pscale);
  auto stored = [&](int k) { return k == kc ? u_first : st_base + (int64_t)((k - kc) / G - 1) * stride; };
  const bool left_end = ts.left_end, right_end = ts.right_end;
  const int lo_t = ts.lo_t, hi_t = ts.hi_t;
  const int qN = ts.qN;
  const int lN = qN / M, jN = uniform(qN % M);
  // points 1 and N-2 (dL/dc1, dL/dcN) when this tile owns them
  const bool own_1 = left_end && 1 < hi_t;
  const int qM = qN - 1;
  const bool own_m = right_end && qM >= lo_t && qM < hi_t && qM >= 1;
  const bool has_edge = ts.has_edge;
  // a tile holding an edge has the longest chain of the launch: its wavefront
  // issues ahead of the plain tiles sharing its SIMD
  if (has_edge) __builtin_amdgcn_s_setprio(2);
  const int b = ts.b, qa = ts.qa;
  const int pa = kRing ? ts.pa : b - 1;
  const int qb = qa + 1;
  const int Q = d + 2;
  F* ha = hist[w][0];
  F* hb = hist[w][1];
  // edly[w][0][k - k0]: u_{lo(b)}(k - dR), the right read of a's last point;
  // edly[w][1][k - k0]: u_{lo(b)-1}(k - dL), the left read of b's first point;
  // pull[w][0][k - k0], pull[w][1][k - k0]: max(k - dL, 0), max(k - dR, 0)
  if (has_edge) {
    // lambda of the edge points for the steps above the launch that a pull
    // of its steps can reach (k+1 .. k+d+1, at most K)
    const int s1 = k0 + steps + d < K ? k0 + steps + d : K;
    for (int s = k0 + steps + lane; s <= s1; s += kWave) {
      ha[s % Q] = LE[((int64_t)s * P + b) * 2];
      hb[s % Q] = LE[((int64_t)s * P + b) * 2 + 1];
    }
    // the delays of the launch's steps and of the d steps above it (whose
    // reads can land on them), and the record values the steps read
    const int kend = k0 + steps - 1 + d < K - 1 ? k0 + steps - 1 + d : K - 1;
    for (int j = lane; j <= kend - k0; j += kWave) {
      const int k = k0 + j;
      const int dL = sched_delay(sched, seed, k, b, 0, P, d);
      const int dR = sched_delay(sched, seed, k, pa, 1, P, d);
      pull[w][0][j] = k - dL > 0 ? k - dL : 0;
      pull[w][1][j] = k - dR > 0 ? k - dR : 0;
      if (j < steps) {
        edly[w][0][j] = E[((int64_t)pull[w][1][j] * P + b) * 2 + 1];
        edly[w][1][j] = E[((int64_t)pull[w][0][j] * P + b) * 2];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  const bool own_a = qa >= lo_t && qa < hi_t, own_b = qb >= lo_t && qb < hi_t;
  double g = 0.0, e1 = 0.0, eN = 0.0;
  const double rd = (double)r;
  // the lane's points whose dL/dr terms this tile sums: its own output
  // points that are updated (not the rod ends)
  uint32_t own_mask = 0;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const int q = q0 + j;
    if (q >= lo_t && q < hi_t && (kRing || (base + q >= 1 && base + q <= N - 2)))
      own_mask |= 1u << j;
  }

  // u(k+1) from u(k) = x, as the forward launches compute it
  auto fwd_step = [&](const F (&x)[M], F (&y)[M], int k) {
#pragma unroll
    for (int j = 0; j < M; ++j) y[j] = x[j];
    lane_step<F, M>(y, from_lower_lane(x[M - 1]), from_upper_lane(x[0]), r);
    if (has_edge) {
      const F ua = read_lane(get_point<F, M>(x, qa % M), qa / M);
      const F ual = qa >= 1 ? read_lane(get_point<F, M>(x, (qa - 1) % M), (qa - 1) / M) : F(0);
      const F ub = qb < L ? read_lane(get_point<F, M>(x, qb % M), qb / M) : F(0);
      const F ubr = qb + 1 < L ? read_lane(get_point<F, M>(x, (qb + 1) % M), (qb + 1) / M) : F(0);
      const F rb = edly[w][0][k - k0], la = edly[w][1][k - k0];
      set_point<F, M>(y, qa % M, lane == qa / M, eq3_step(ual, ua, rb, r));
      if (qb < L) set_point<F, M>(y, qb % M, lane == qb / M, eq3_step(la, ub, ubr, r));
    }
    if (left_end) y[0] = (lane == 0) ? c1 : y[0];
    if (right_end) set_point<F, M>(y, jN, lane == lN, cN);
  };

  // lambda(k) from lambda(k+1) (in l) and u(k) = uc
  auto bwd_step = [&](const F (&uc)[M], int k) {
    F la1 = F(0), lal1 = F(0), lb1 = F(0), lbr1 = F(0), ua = F(0), ub = F(0);
    if (has_edge) {
      la1 = read_lane(get_point<F, M>(l, qa % M), qa / M);
      ua = read_lane(get_point<F, M>(uc, qa % M), qa / M);
      if (qa >= 1) lal1 = read_lane(get_point<F, M>(l, (qa - 1) % M), (qa - 1) / M);
      if (qb < L) {
        lb1 = read_lane(get_point<F, M>(l, qb % M), qb / M);
        ub = read_lane(get_point<F, M>(uc, qb % M), qb / M);
      }
      if (qb + 1 < L) lbr1 = read_lane(get_point<F, M>(l, (qb + 1) % M), (qb + 1) / M);
    }
    if (own_1) e1 += rd * (double)read_lane(l[1 % M], 1 / M);
    if (own_m) eN += rd * (double)read_lane(get_point<F, M>(l, qM % M), qM / M);
    // dL/dr with the plain Laplacians over the tile's own points: the lane's
    // terms of this step summed in the state precision (two chains), then
    // added to the double total
    const F ul = from_lower_lane(uc[M - 1]), ur = from_upper_lane(uc[0]);
    {
      F acc[2] = {F(0), F(0)};
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const F uL = j > 0 ? uc[j - 1] : ul, uR = j + 1 < M ? uc[j + 1] : ur;
        const F lm = ((own_mask >> j) & 1u) ? l[j] : F(0);
        acc[j & 1] = fma_of(lm, fma_of(F(-2), uc[j], uL + uR), acc[j & 1]);
      }
      g += (double)(acc[0] + acc[1]);
    }
    // the plain transpose step of every point
    {
      const F left = from_lower_lane(l[M - 1]);
      const F right = from_upper_lane(l[0]);
      F prev = left;
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const F c = l[j];
        const F nx = j + 1 < M ? l[j + 1] : right;
        l[j] = fma_of(r, fma_of(F(-2), c, prev + nx), c);
        prev = c;
      }
    }
    if (has_edge) {
      const int kmax = k + d < K - 1 ? k + d : K - 1;
      // the delayed Laplacians of the edge points, as corrections of the plain ones
      const F uRd = edly[w][0][k - k0], uLd = edly[w][1][k - k0];
      if (lane == 0) {
        if (own_a) g += (double)la1 * ((double)uRd - (double)ub);
        if (own_b) g += (double)lb1 * ((double)uLd - (double)ua);
      }
      // point a: the pulls of b's left reads first, then its left neighbour;
      // point b: its right neighbour first, then the pulls of a's right reads.
      // Lane j looks at step kk = k + j (a chunk of up to 64 steps at a time);
      // the hits are added in order of kk.
      F nba = F(0);
      F nbb = F(0);
      nbb += lbr1;
      for (int c = k; c <= kmax; c += kWave) {
        const int kk = c + lane;
        const bool in = kk <= kmax;
        const bool hit_a = in && pull[w][0][kk - k0] == k;
        const bool hit_b = in && pull[w][1][kk - k0] == k;
        const F vb = (in && kk > k) ? hb[(kk + 1) % Q] : lb1;  // lambda_b(kk+1)
        const F va = (in && kk > k) ? ha[(kk + 1) % Q] : la1;  // lambda_a(kk+1)
        for (uint64_t m = __ballot(hit_a); m; m &= m - 1)
          nba += read_lane(vb, __builtin_ctzll(m));
        for (uint64_t m = __ballot(hit_b); m; m &= m - 1)
          nbb += read_lane(va, __builtin_ctzll(m));
      }
      nba += lal1;
      const F na = fma_of(r, fma_of(F(-2), la1, nba), la1);
      const F nb = fma_of(r, fma_of(F(-2), lb1, nbb), lb1);
      set_point<F, M>(l, qa % M, lane == qa / M, na);
      if (qb < L) set_point<F, M>(l, qb % M, lane == qb / M, nb);
      if (lane == 0) {
        ha[k % Q] = na;
        hb[k % Q] = nb;
        if (own_a) LE[((int64_t)k * P + b) * 2] = na;
        if (own_b) LE[((int64_t)k * P + b) * 2 + 1] = nb;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // lambda of the fixed ends stays 0
    if (left_end) l[0] = (lane == 0) ? F(0) : l[0];
    if (right_end) set_point<F, M>(l, jN, lane == lN, F(0));
  };

  // groups of up to G steps from the top: the stored state at the group's
  // bottom, the states above it recomputed, then the transpose steps
  // downwards; the next group's stored state is loaded into the top state's
  // registers once its step is done (three steps of work hide the load)
  const int ktop = k0 + steps - 1;
  int k4 = kc + (ktop - kc) / G * G;
  F s0[M], s1[M], s2[M], s3[M];
  load_tile<F, M, kRing>(s0, stored(k4), base, q0, L, N, aligned != 0);
  for (int k = ktop; k >= k0;) {
    const int k4n = k4 - G;
    const int n = k - k4 + 1;
    static_assert(G == 4, "the group is written out for four states");
    if (n >= 2) fwd_step(s0, s1, k4);
    if (n >= 3) fwd_step(s1, s2, k4 + 1);
    if (n >= 4) fwd_step(s2, s3, k4 + 2);
    if (n >= 4) bwd_step(s3, k4 + 3);
    if (k4n >= k0) load_tile<F, M, kRing>(s3, stored(k4n), base, q0, L, N, aligned != 0);
    if (n >= 3) bwd_step(s2, k4 + 2);
    if (n >= 2) bwd_step(s1, k4 + 1);
    bwd_step(s0, k4);
    k = k4 - 1;
    k4 = k4n;
    if (k >= k0) {
#pragma unroll
      for (int j = 0; j < M; ++j) s0[j] = s3[j];
    }
  }
  store_points<F, M>(l, lam_out, base + q0, q0, lo_t, hi_t, aligned != 0 && base >= 0);
  for (int off = kWave / 2; off > 0; off >>= 1) g += __shfl_xor(g, off, kWave);
  if (lane == 0) {
    part[t] += g;
    if (own_1) ends[0] += e1;
    if (own_m) ends[1] += eN;
  }
}

// lambda(k) from lambda(k+1) and u(k) (the transpose of the step above), the
// dL/dr term of step k summed per workgroup into part[blockIdx.x], and the
// dL/dc1, dL/dcN terms of step k added to ends[0], ends[1].  Each workgroup
// owns its partial slot and the grid is the same for every step, so the sums
// run in a fixed order.
template <typename F, bool kRing>
__global__ __launch_bounds__(kThreads) void async_adjoint_step_kernel(
    const F* __restrict__ lam1, F* __restrict__ lam0, const F* __restrict__ u,
    const F* __restrict__ E, F* __restrict__ LE, const int64_t* __restrict__ lo, int64_t N,
    int P, int k, int K, int d, uint64_t seed, int sched, F r, double pscale,
    double* __restrict__ part, double* __restrict__ ends, int aligned) {
  __shared__ double red[kThreads / kWave];
  const int64_t i0 = ((int64_t)blockIdx.x * kThreads + threadIdx.x) * kPts;
  double g = 0.0;
  if (i0 < N) {
    F l[kPts], c[kPts], out[kPts];
    load_points<F, kPts>(l, lam1, i0, N, aligned != 0);
    load_points<F, kPts>(c, u, i0, N, aligned != 0);
    const F lb = i0 >= 1 ? lam1[i0 - 1] : F(0), la = i0 + kPts < N ? lam1[i0 + kPts] : F(0);
    const F ub = i0 >= 1 ? u[i0 - 1] : F(0), ua = i0 + kPts < N ? u[i0 + kPts] : F(0);
    EdgeScan<kRing> es = edge_scan<kRing>(i0, lo, P, pscale);
    const bool plain = es.none_in(i0, kPts, P) && i0 >= 2 && i0 + kPts <= N - 2;
    if (plain) {
      // no edge, no end and no end neighbour among the group's points
#pragma unroll
      for (int j = 0; j < kPts; ++j) {
        const F uL = j > 0 ? c[j - 1] : ub, uR = j + 1 < kPts ? c[j + 1] : ua;
        const F nb = (j > 0 ? l[j - 1] : lb) + (j + 1 < kPts ? l[j + 1] : la);
        g += (double)l[j] * ((double)uL + (double)uR - 2.0 * (double)c[j]);
        out[j] = fma_of(r, fma_of(F(-2), l[j], nb), l[j]);
      }
    } else {
      const int kmax = k + d < K - 1 ? k + d : K - 1;
#pragma unroll
      for (int j = 0; j < kPts; ++j) {
        const int64_t i = i0 + j;
        out[j] = F(0);
        if (i >= N || (!kRing && (i < 1 || i > N - 2))) continue;
        es.to(i, lo, P);
        const int p = es.p;
        const int eL = es.left_edge(), eR = es.right_edge(P);
        const bool first = es.first(i), last = es.last(i, P);
        const F l1 = l[j];
        // dL/dr: lambda_i(k+1) times the Laplacian the forward step used
        F uL = j > 0 ? c[j - 1] : ub, uR = j + 1 < kPts ? c[j + 1] : ua;
        if (first) {
          const int dl = sched_delay(sched, seed, k, p, 0, P, d);
          uL = E[((int64_t)(k - dl > 0 ? k - dl : 0) * P + eL) * 2];
        }
        if (last) {
          const int dr = sched_delay(sched, seed, k, p, 1, P, d);
          uR = E[((int64_t)(k - dr > 0 ? k - dr : 0) * P + eR) * 2 + 1];
        }
        g += (double)l1 * ((double)uL + (double)uR - 2.0 * (double)c[j]);
        // the neighbours' reads of u_i(k) (on the ring every neighbour is updated)
        F nb = F(0);
        if (kRing || i + 1 <= N - 2) {
          if (last) {  // the next point opens the next subdomain and read u_i with its left delays
            const int pn = p + 1 == P ? 0 : p + 1;
            for (int kk = k; kk <= kmax; ++kk) {
              const int dl = sched_delay(sched, seed, kk, pn, 0, P, d);
              if ((kk - dl > 0 ? kk - dl : 0) == k)
                nb += LE[((int64_t)(kk + 1) * P + eR) * 2 + 1];
            }
          } else {
            nb += j + 1 < kPts ? l[j + 1] : la;
          }
        }
        if (kRing || i - 1 >= 1) {
          if (first) {  // the previous point closes the previous subdomain and read u_i with its right delays
            const int pp = p == 0 ? P - 1 : p - 1;
            for (int kk = k; kk <= kmax; ++kk) {
              const int dr = sched_delay(sched, seed, kk, pp, 1, P, d);
              if ((kk - dr > 0 ? kk - dr : 0) == k) nb += LE[((int64_t)(kk + 1) * P + eL) * 2];
            }
          } else {
            nb += j > 0 ? l[j - 1] : lb;
          }
        }
        const F lnew = fma_of(r, fma_of(F(-2), l1, nb), l1);
        out[j] = lnew;
        if (first) LE[((int64_t)k * P + eL) * 2 + 1] = lnew;
        if (last) LE[((int64_t)k * P + eR) * 2] = lnew;
        if (!kRing && i == 1) ends[0] += (double)r * (double)l1;
        if (!kRing && i == N - 2) ends[1] += (double)r * (double)l1;
      }
    }
    store_points<F, kPts>(out, lam0, i0, 0, 0, (int)(N - i0 < kPts ? N - i0 : kPts),
                          aligned != 0);
  }
  // workgroup sum of g in a fixed order: lanes by a butterfly, then wavefronts
  for (int off = kWave / 2; off > 0; off >>= 1) g += __shfl_xor(g, off, kWave);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == 0) red[wave] = g;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kThreads / kWave; ++w) s += red[w];
    part[blockIdx.x] += s;
  }
}

// grad_c1 = gK[0] + ends[0], grad_cN = gK[N-1] + ends[1].
template <typename F>
__global__ void adjoint_ends_kernel(const F* __restrict__ gK, int64_t N,
                                    const double* __restrict__ ends, double* grad_c1,
                                    double* grad_cN, int ring) {
  if (threadIdx.x == 0) {
    *grad_c1 = ring ? 0.0 : (double)gK[0] + ends[0];
    *grad_cN = ring ? 0.0 : (double)gK[N - 1] + ends[1];
  }
}

__global__ void zero_f64_kernel(double* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

bool is_aligned16(const void* q) { return ((uintptr_t)q & 15u) == 0; }
int aligned_pair(const void* a, const void* b, int64_t) {
  return is_aligned16(a) && is_aligned16(b);
}

}  // namespace

int64_t async_adjoint_blocks(int64_t N) {
  return (N + (int64_t)kThreads * kPts - 1) / ((int64_t)kThreads * kPts);
}

hipError_t launch_async_partition(int64_t* lo, int64_t N, int P, hipStream_t s) {
  hipLaunchKernelGGL(partition_kernel, dim3((unsigned)((P + 1 + 255) / 256)), dim3(256), 0, s, lo,
                     N, P);
  return hipGetLastError();
}

hipError_t launch_async_edges(int dtype, const void* u, void* Ek, const int64_t* lo, int P,
                              int64_t N, int ring, hipStream_t s) {
  if (P < 2) return hipSuccess;
  const dim3 grid((unsigned)((P + 255) / 256));
  if (dtype == 0)
    hipLaunchKernelGGL(edges_from_state_kernel<float>, grid, dim3(256), 0, s, (const float*)u,
                       (float*)Ek, lo, P, N, ring);
  else
    hipLaunchKernelGGL(edges_from_state_kernel<double>, grid, dim3(256), 0, s, (const double*)u,
                       (double*)Ek, lo, P, N, ring);
  return hipGetLastError();
}

template <typename F, bool kRing>
static void lockstep_launch(const AsyncAdjStep& a, const void* cur, void* nxt, int k, int record,
                            hipStream_t s) {
  hipLaunchKernelGGL((async_lockstep_kernel<F, kRing>), dim3((unsigned)async_adjoint_blocks(a.N)),
                     dim3(kThreads), 0, s, (const F*)cur, (F*)nxt, (F*)a.E, a.lo, a.N, a.P, k,
                     a.d, a.seed, a.sched, (F)a.r, (F)a.c1, (F)a.cN, (double)a.P / (double)a.N, record,
                     aligned_pair(cur, nxt, a.N));
}

hipError_t launch_async_lockstep(const AsyncAdjStep& a, const void* cur, void* nxt, int k,
                                 int record, hipStream_t s) {
  if (a.dtype == 0)
    a.ring ? lockstep_launch<float, true>(a, cur, nxt, k, record, s)
           : lockstep_launch<float, false>(a, cur, nxt, k, record, s);
  else
    a.ring ? lockstep_launch<double, true>(a, cur, nxt, k, record, s)
           : lockstep_launch<double, false>(a, cur, nxt, k, record, s);
  return hipGetLastError();
}

bool async_tiled_applies(int64_t N, int P, int d) {
  return d + 2 <= kHistQ && (P == 1 || N / P > (int64_t)kWave * kTileM);
}

int async_tiled_depth() { return kTileT; }

template <typename F, bool kRing>
static void lockstep_tiled_launch(const AsyncAdjStep& a, const TileGeom& g, const void* in,
                                  void* out, void* states, int64_t stride, int kc, int k0,
                                  int steps, int record, int aligned, hipStream_t s) {
  hipLaunchKernelGGL((async_lockstep_tiled_kernel<F, kRing>),
                     dim3((unsigned)((g.tiles_per_rod + kAdjWaves - 1) / kAdjWaves)),
                     dim3(kAdjWaves * kWave), 0, s, (const F*)in, (F*)out, (F*)states, stride,
                     kc, (F*)a.E, a.ord_lock, a.N, a.P, k0, steps, a.d, a.seed, a.sched, (F)a.r, (F)a.c1,
                     (F)a.cN, g.tiles_per_rod, g.H, (double)a.P / (double)a.N, record, aligned);
}

hipError_t launch_async_lockstep_tiled(const AsyncAdjStep& a, const void* in, void* out,
                                       void* states, int64_t stride, int kc, int k0, int steps,
                                       int record, hipStream_t s) {
  const TileGeom g = a.ring ? ring_geometry(a.dtype, kTileM, kTileT, a.N)
                            : tile_geometry(a.dtype, kTileM, kTileT, a.N);
  if (steps < 1 || steps > g.H || steps > kTileT || g.tiles_per_rod <= 0 || g.Wout <= 0 ||
      !async_tiled_applies(a.N, a.P, a.d) || (a.ring && a.P < 2) || (states && k0 < kc))
    return hipErrorInvalidValue;
  const int aligned = is_aligned16(in) && (!out || is_aligned16(out)) &&
                      (!states || is_aligned16(states)) && stride % 4 == 0;
  if (a.dtype == 0)
    a.ring ? lockstep_tiled_launch<float, true>(a, g, in, out, states, stride, kc, k0, steps,
                                                record, aligned, s)
           : lockstep_tiled_launch<float, false>(a, g, in, out, states, stride, kc, k0, steps,
                                                 record, aligned, s);
  else
    a.ring ? lockstep_tiled_launch<double, true>(a, g, in, out, states, stride, kc, k0, steps,
                                                 record, aligned, s)
           : lockstep_tiled_launch<double, false>(a, g, in, out, states, stride, kc, k0, steps,
                                                  record, aligned, s);
  return hipGetLastError();
}

int async_tiled_store_every() { return kStoreEvery; }

hipError_t launch_async_tiled_order(const AsyncAdjStep& a, int* ord_lock, int* ord_adj,
                                    hipStream_t s) {
  if (!async_tiled_applies(a.N, a.P, a.d) || (a.ring && a.P < 2)) return hipErrorInvalidValue;
  const double pscale = (double)a.P / (double)a.N;
  for (int which = 0; which < 2; ++which) {
    const int T = which == 0 ? kTileT : kAdjT;
    const TileGeom g = a.ring ? ring_geometry(a.dtype, kTileM, T, a.N)
                              : tile_geometry(a.dtype, kTileM, T, a.N);
    if (g.tiles_per_rod <= 0 || g.Wout <= 0) return hipErrorInvalidValue;
    int* ord = which == 0 ? ord_lock : ord_adj;
    if (a.ring)
      hipLaunchKernelGGL(tile_order_kernel<true>, dim3(1), dim3(256), 0, s, ord, g.tiles_per_rod,
                         kWave * kTileM, g.H, a.N, a.P, pscale);
    else
      hipLaunchKernelGGL(tile_order_kernel<false>, dim3(1), dim3(256), 0, s, ord, g.tiles_per_rod,
                         kWave * kTileM, g.H, a.N, a.P, pscale);
  }
  return hipGetLastError();
}

int64_t async_tiled_tiles(int dtype, int64_t N) {
  return std::max(tile_geometry(dtype, kTileM, kAdjT, N).tiles_per_rod,
                  ring_geometry(dtype, kTileM, kAdjT, N).tiles_per_rod);
}

template <typename F, bool kRing>
static void adjoint_tiled_launch(const AsyncAdjStep& a, const TileGeom& g, const void* lam_in,
                                 void* lam_out, const void* u_first, const void* st_base,
                                 int64_t stride, int kc, int k0, int steps, int aligned,
                                 hipStream_t s) {
  hipLaunchKernelGGL((async_adjoint_tiled_kernel<F, kRing>),
                     dim3((unsigned)((g.tiles_per_rod + kAdjWaves - 1) / kAdjWaves)),
                     dim3(kAdjWaves * kWave), 0, s, (const F*)lam_in, (F*)lam_out,
                     (const F*)u_first, (const F*)st_base, stride, kc, (const F*)a.E,
                     (F*)a.LE, a.ord_adj, a.N, a.P, k0, steps, a.K, a.d, a.seed, a.sched, (F)a.r, (F)a.c1,
                     (F)a.cN, g.tiles_per_rod, g.H, (double)a.P / (double)a.N, a.part, a.ends,
                     aligned);
}

hipError_t launch_async_adjoint_tiled(const AsyncAdjStep& a, const void* lam_in, void* lam_out,
                                      const void* u_first, const void* st_base, int64_t stride,
                                      int kc, int k0, int steps, hipStream_t s) {
  const TileGeom g = a.ring ? ring_geometry(a.dtype, kTileM, kAdjT, a.N)
                            : tile_geometry(a.dtype, kTileM, kAdjT, a.N);
  if (steps < 1 || steps > kTileT || steps + kStoreEvery - 1 > g.H || g.tiles_per_rod <= 0 ||
      g.Wout <= 0 || !async_tiled_applies(a.N, a.P, a.d) || (a.ring && a.P < 2) || k0 < kc ||
      (k0 - kc) % kStoreEvery != 0)
    return hipErrorInvalidValue;
  const int aligned = is_aligned16(lam_in) && is_aligned16(lam_out) && is_aligned16(u_first) &&
                      is_aligned16(st_base) && stride % 4 == 0;
  if (a.dtype == 0)
    a.ring ? adjoint_tiled_launch<float, true>(a, g, lam_in, lam_out, u_first, st_base, stride,
                                               kc, k0, steps, aligned, s)
           : adjoint_tiled_launch<float, false>(a, g, lam_in, lam_out, u_first, st_base, stride,
                                                kc, k0, steps, aligned, s);
  else
    a.ring ? adjoint_tiled_launch<double, true>(a, g, lam_in, lam_out, u_first, st_base, stride,
                                                kc, k0, steps, aligned, s)
           : adjoint_tiled_launch<double, false>(a, g, lam_in, lam_out, u_first, st_base, stride,
                                                 kc, k0, steps, aligned, s);
  return hipGetLastError();
}

template <typename F, bool kRing>
static void adjoint_step_launch(const AsyncAdjStep& a, const void* lam1, void* lam0,
                                const void* u, int k, hipStream_t s) {
  hipLaunchKernelGGL((async_adjoint_step_kernel<F, kRing>),
                     dim3((unsigned)async_adjoint_blocks(a.N)), dim3(kThreads), 0, s,
                     (const F*)lam1, (F*)lam0, (const F*)u, (const F*)a.E, (F*)a.LE, a.lo, a.N,
                     a.P, k, a.K, a.d, a.seed, a.sched, (F)a.r, (double)a.P / (double)a.N, a.part, a.ends,
                     aligned_pair(lam1, lam0, a.N) && is_aligned16(u));
}

hipError_t launch_async_adjoint_step(const AsyncAdjStep& a, const void* lam1, void* lam0,
                                     const void* u, int k, hipStream_t s) {
  if (a.dtype == 0)
    a.ring ? adjoint_step_launch<float, true>(a, lam1, lam0, u, k, s)
           : adjoint_step_launch<float, false>(a, lam1, lam0, u, k, s);
  else
    a.ring ? adjoint_step_launch<double, true>(a, lam1, lam0, u, k, s)
           : adjoint_step_launch<double, false>(a, lam1, lam0, u, k, s);
  return hipGetLastError();
}

hipError_t launch_async_adjoint_ends(int dtype, const void* gK, int64_t N, const double* ends,
                                     double* grad_c1, double* grad_cN, int ring, hipStream_t s) {
  if (dtype == 0)
    hipLaunchKernelGGL(adjoint_ends_kernel<float>, dim3(1), dim3(64), 0, s, (const float*)gK, N,
                       ends, grad_c1, grad_cN, ring);
  else
    hipLaunchKernelGGL(adjoint_ends_kernel<double>, dim3(1), dim3(64), 0, s, (const double*)gK,
                       N, ends, grad_c1, grad_cN, ring);
  return hipGetLastError();
}

hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(zero_f64_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace heat1d
