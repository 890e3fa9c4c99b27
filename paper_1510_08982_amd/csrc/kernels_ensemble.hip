// kernels_ensemble.hip -- an ensemble of emulated asynchronous runs of equal
// rods in one launch (Section 5, Fig. 3: many runs of the same rod whose
// trajectories differ only through their random communication delays), with
// Dirichlet ends or on the periodic ring of Section 5.3 (Fig. 6).
//
// One workgroup of eight wavefronts per member.
// In the emulated mode the result
// of Eq.4 is a fixed function of the seed, so the subdomains of a member need
// no real concurrency: the workgroup advances all P subdomains together, one
// barrier per step, and keeps the last d+2 states of the rod in LDS (the d+1
// states a delayed read may use plus the one being written), so a subdomain
// edge can read its neighbour at any age 0..d.
//
// The delays do not depend on the state.  Drawing them (two SplitMix64
// evaluations each) costs far more than the update itself, and a rod of the
// paper's size has fewer points than the workgroup has lanes, so the draws of
// step k+1 are spread over every thread of the workgroup during step k and
// left in a small LDS table (one byte per subdomain edge, two rows used in
// turn); the update of step k reads its delays from the row filled during step
// k-1, issuing those reads before the draws so that they complete meanwhile.
//
// The 2-norm of the state is summed in double from the values each thread has
// just computed, reduced per wavefront with DPP row operations and across
// wavefronts by thread 0 during the next step; the partials alternate between
// two LDS rows so that no second barrier is needed.
#include <algorithm>

#include "heat1d_device.h"
#include "heat1d_ensemble.h"

namespace heat1d {

// Forward: eight wavefronts per member; the delay draws go to the highest
// threads first, so on a rod with fewer points than threads the wavefronts
// that update points and those that draw are mostly different ones and
// share each SIMD's issue slots instead of running back to back.
constexpr int kFwdWaves = 8;
constexpr int kFwdThreads = kFwdWaves * kWave;
// Adjoint: the same shape, draws likewise on the highest threads.
constexpr int kAdjWaves = 8;
constexpr int kAdjThreads = kAdjWaves * kWave;
constexpr int32_t kEdgeLeft = 0x40000000, kEdgeRight = (int32_t)0x80000000u;

static inline int64_t round8(int64_t x) { return (x + 7) & ~int64_t(7); }

int64_t ensemble_lds_bytes(int dtype, int64_t N, int64_t P, int d) {
  const int64_t es = dtype == 0 ? 4 : 8;
  const int64_t table = d > 0 ? round8(4 * P) : 0;  // no draws when every delay is 0
  return round8((int64_t)(d + 2) * N * es) + table + 2 * kFwdWaves * 8;
}

struct EnsDev {
  const void* u0;
  void* uK;     // or nullptr
  void* traj;   // every state u(0..K) of every member, or nullptr
  const uint64_t* seeds;
  double* norms;
  int64_t nobs;
  int32_t N, P, K, d, Q, every;
  int32_t ring_bytes, dtab_bytes;
  double r, c1, cN;
  void* snaps;  // the states at snap_steps[0..nsnap) of every member, or nullptr
  int32_t nsnap;
  int32_t snap_steps[kEnsembleMaxSnaps];
};

// DPP move of a double with a row mask (rows outside it receive 0).
template <int Ctrl, int RowMask>
__device__ __forceinline__ double dpp_rows(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), Ctrl, RowMask, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), Ctrl, RowMask, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the wavefront (all 64 lanes active), complete in lane 63:
// butterflies inside each row of 16 lanes, then rows 1 and 3 add the sum of the
// row below, and rows 2 and 3 the sum of rows 0 and 1.  A fixed order, so the
// same bits on every run.
__device__ __forceinline__ double wave_sum_to_last(double v) {
  v += dpp<0xB1>(v);             // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);             // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);            // row_half_mirror
  v += dpp<0x140>(v);            // row_mirror
  v += dpp_rows<0x142, 0xA>(v);  // row_bcast:15
  v += dpp_rows<0x143, 0xC>(v);  // row_bcast:31
  return v;
}

// Subdomain of point i (the largest p with floor(p N / P) <= i), plus
// kEdgeLeft if i is the first point of p and kEdgeRight if it is the last: the
// points whose neighbour across a subdomain boundary is read with a delay.  On
// the Dirichlet rod subdomain 0 has no left and subdomain P-1 no right
// neighbour; on the ring (kRing) every subdomain has both when P > 1.
template <bool kRing>
__device__ __forceinline__ int32_t point_meta(int64_t i, int64_t N, int64_t P) {
  const int64_t p = ((i + 1) * P + N - 1) / N - 1;
  const int64_t lo = p * N / P, hi = (p + 1) * N / P;
  uint32_t m = (uint32_t)p;
  if ((kRing ? P > 1 : p > 0) && i == lo) m |= (uint32_t)kEdgeLeft;
  if ((kRing ? P > 1 : p < P - 1) && i == hi - 1) m |= (uint32_t)kEdgeRight;
  return (int32_t)m;
}

// Delay of the emulated schedule with counter c = ((k P + p) << 1) | side
// (= 2kP + q for the table entry q = 2p + side): the value the schedule's
// definition gives, with the top-word product taken directly.
__device__ __forceinline__ int delay_at(uint64_t seed, uint64_t c, uint32_t dp1) {
  const uint64_t x = sm64(seed ^ sm64(c));
  return (int)__umulhi((uint32_t)(x >> 32), dp1);
}

// Ring slot of step k - dl, given the slot kq of step k (steps before 0 read
// step 0, which stays in slot 0 until step d+2 is written).
__device__ __forceinline__ int delayed_slot(int k, int kq, int dl, int Q) {
  return k < dl ? 0 : (kq >= dl ? kq - dl : kq - dl + Q);
}

// kRing: the periodic boundary of Section 5.3 (all N points updated, point 0
// and point N-1 neighbours); otherwise the Dirichlet rod (points 1..N-2).
template <typename F, int PPT, bool kRing>
__global__ __launch_bounds__(kFwdThreads) void ensemble_kernel(EnsDev a) {
  extern __shared__ __align__(16) unsigned char smem[];
  F* ring = reinterpret_cast<F*>(smem);
  uint8_t* dtab = smem + a.ring_bytes;  // two rows of 2P delays: entry 2p + side
  double* wpart = reinterpret_cast<double*>(smem + a.ring_bytes + a.dtab_bytes);
  const int N = a.N, Q = a.Q, P = a.P, d = a.d;
  const int tid = threadIdx.x;
  const int wave = tid / kWave, lane = tid % kWave;
  const int64_t e = blockIdx.x;
  const uint64_t seed = a.seeds[e];
  const F* __restrict__ u0 = static_cast<const F*>(a.u0) + e * N;
  const F c1 = (F)a.c1, cN = (F)a.cN, r = (F)a.r;
  double* __restrict__ norms = a.norms ? a.norms + e * a.nobs : nullptr;
  // the trajectory of this member: state k at traj + k*N (updated points only)
  F* __restrict__ traj = a.traj ? static_cast<F*>(a.traj) + e * (int64_t)(a.K + 1) * N : nullptr;
  // the states this member reports (Section 5.1, Fig. 2): snapshot j at
  // snaps + j*N, written by the threads that compute its points
  F* __restrict__ snaps =
      a.snaps ? static_cast<F*>(a.snaps) + e * (int64_t)a.nsnap * N : nullptr;
  int si = 0;  // next snapshot
  auto snap_ends = [&](F* dst) {
    if (!kRing && tid == 0) {
      dst[0] = c1;
      dst[N - 1] = cN;
    }
  };
  const double ends_sq = kRing ? 0.0 : (double)c1 * (double)c1 + (double)cN * (double)cN;
  const int first = kRing ? 0 : 1, last = kRing ? N : N - 1;  // updated points [first, last)
  const int ndraw = d > 0 ? 2 * P : 0;  // with d = 0 every delay is 0: no table
  const uint32_t dp1 = (uint32_t)d + 1;
  const uint64_t two_p = 2 * (uint64_t)P;

  // this thread's points first + tid + j*nt and their subdomain flags; the
  // delays of step 0 in row 0 of the table
  int32_t mt[PPT];
  double acc = 0.0;
  F* snap0 = (snaps && a.nsnap > 0 && a.snap_steps[0] == 0) ? snaps : nullptr;
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int i = first + tid + j * kFwdThreads;
    mt[j] = i < last ? point_meta<kRing>(i, N, P) : 0;
    if (i < last) {
      const F v = u0[i];
      ring[i] = v;
      if (traj) traj[i] = v;
      if (snap0) snap0[i] = v;
      acc = __builtin_fma((double)v, (double)v, acc);
    }
  }
  if (snap0) {
    snap_ends(snap0);
    si = 1;
  }
  for (int q = kFwdThreads - 1 - tid; q < ndraw; q += kFwdThreads)
    dtab[q] = (uint8_t)delay_at(seed, (uint64_t)q, dp1);
  // the Dirichlet ends of every slot (no step writes them)
  if (!kRing) {
    for (int s = tid; s < Q; s += kFwdThreads) {
      ring[s * N] = c1;
      ring[s * N + N - 1] = cN;
    }
  }
  // An observation's wavefront partials are combined by thread 0 during the
  // following step, after that step's own work: they were published by the
  // barrier in between, and their row is not written again before the next
  // barrier.
  int pend = -1;  // norm index waiting in row prow, or -1
  int prow = 0;
  int obs_in = a.every;  // steps to the next observation
  auto combine = [&]() {
    // by a thread of the third wavefront: on a rod shorter than 128 points it
    // neither updates points nor draws delays, so the sum is off the path
    // that the other wavefronts wait for at the barrier
    if (tid == 2 * kWave) {
      const double* w = wpart + prow;
      norms[pend] = sqrt(ends_sq + (((w[0] + w[1]) + (w[2] + w[3])) + ((w[4] + w[5]) + (w[6] + w[7]))));
    }
    pend = -1;
  };
  // wavefronts that own no point skip the reduction (their partial is 0)
  const bool has_points = first + wave * kWave < last;
  if (norms) {
    if (has_points) acc = wave_sum_to_last(acc);
    if (lane == kWave - 1) wpart[kFwdWaves + wave] = acc;
    pend = 0;
    prow = kFwdWaves;
  }
  __syncthreads();

  int kq = 0;  // slot holding step k
  uint64_t cbase = two_p;  // 2 (k+1) P: the counter base of the next step's draws
  for (int k = 0; k < a.K; ++k) {
    const int nq = kq + 1 == Q ? 0 : kq + 1;
    const F* cur = ring + kq * N;
    F* nxt = ring + nq * N;
    const uint8_t* drow = dtab + (k & 1) * ndraw;
    // this step's delays, read before the next step's are drawn
    int dlL[PPT], dlR[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int pp = 2 * (mt[j] & 0x3fffffff);
      dlL[j] = (ndraw && (mt[j] & kEdgeLeft)) ? drow[pp] : 0;
      dlR[j] = (ndraw && (mt[j] & kEdgeRight)) ? drow[pp + 1] : 0;
    }
    {
      uint8_t* wrow = dtab + ((k + 1) & 1) * ndraw;
      for (int q = kFwdThreads - 1 - tid; q < ndraw; q += kFwdThreads)
        wrow[q] = (uint8_t)delay_at(seed, cbase + (uint64_t)q, dp1);
      cbase += two_p;
    }
    acc = 0.0;
    F* snap = (snaps && si < a.nsnap && a.snap_steps[si] == k + 1) ? snaps + (int64_t)si * N
                                                                     : nullptr;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int i = first + tid + j * kFwdThreads;
      if (i < last) {
        const int il = (kRing && i == 0) ? N - 1 : i - 1;
        const int ir = (kRing && i == N - 1) ? 0 : i + 1;
        const F* lsrc = (mt[j] & kEdgeLeft) ? ring + delayed_slot(k, kq, dlL[j], Q) * N : cur;
        const F* rsrc = (mt[j] & kEdgeRight) ? ring + delayed_slot(k, kq, dlR[j], Q) * N : cur;
        const F v = eq3_step(lsrc[il], cur[i], rsrc[ir], r);
        nxt[i] = v;
        if (traj) traj[(int64_t)(k + 1) * N + i] = v;
        if (snap) snap[i] = v;
        acc = __builtin_fma((double)v, (double)v, acc);
      }
    }
    if (snap) {
      snap_ends(snap);
      ++si;
    }
    if (pend >= 0) combine();
    if (norms && --obs_in == 0) {
      obs_in = a.every;
      const int row = (k & 1) * kFwdWaves;
      if (has_points) acc = wave_sum_to_last(acc);
      if (lane == kWave - 1) wpart[row + wave] = acc;
      pend = (k + 1) / a.every;
      prow = row;
    }
    __syncthreads();
    kq = nq;
  }
  if (pend >= 0) combine();

  if (a.uK) {
    F* __restrict__ out = static_cast<F*>(a.uK) + e * N;
    const F* fin = ring + kq * N;
    for (int i = tid; i < N; i += kFwdThreads) out[i] = fin[i];
  }
}

// ---------------------------------------------------------------------------
// Adjoint of one member's emulated asynchronous run (Dirichlet ends), derived
// from Eq.4.  For a fixed schedule the step is linear in the states it reads,
// so reverse mode sends, for every point i and step k, (1-2r) lambda_i(k+1) to
// u_i(k) and r lambda_i(k+1) to each neighbour value the step read, at the
// step that read landed on (the delay schedule reversed):
//   lambda_j(k) = lambda_j(k+1) + r (nb - 2 lambda_j(k+1)),
//   nb = the lambda_{j+-1}(k'+1) of every step k' at which neighbour j+-1
//        read point j's value of step k,
// the same three instructions as a forward step.  A read inside a subdomain,
// or across an edge with delay 0, lands on its own step: the neighbour's
// lambda(k+1) is read directly.  A delayed read lands on an earlier step s:
// the reader adds its lambda into an LDS accumulator for (s, target) -- one
// row per landing step, one accumulator per direction, so each has a single
// writer per step -- which the target point adds in (and clears) when the
// reverse sweep reaches step s.  Every point does a fixed amount of LDS work
// per step whatever d is.  dL/dr sums lambda_j(k+1) (u_{j-1}(sL) + u_{j+1}(sR)
// - 2 u_j(k)) over the reads of the forward step; dL/dc1 and dL/dcN the
// r lambda(k+1) of points 1 and N-2 (their reads of the ends) plus the end
// entries of gK.  The forward states come back from the trajectory the forward
// launch stored; the workgroup keeps the d+1 states a step reads plus the
// next one in an LDS ring and d+2 rows of delays (the draws of step k-1 are
// spread over the threads during step k).
struct EnsAdjDev {
  const void* traj;  // member e: E x (K+1) states of N points (interior points valid)
  const void* gK;
  const uint64_t* seeds;
  void* grad_u0;
  double* grad_r;
  double* grad_c1;
  double* grad_cN;
  int32_t N, P, K, d;
  int32_t uring_bytes, lring_bytes, pend_bytes, dtab_bytes;
  double r, c1, cN;
};

int64_t ensemble_adjoint_lds_bytes(int dtype, int64_t N, int64_t P, int d) {
  const int64_t es = dtype == 0 ? 4 : 8;
  const int64_t table = d > 0 ? round8((int64_t)(d + 2) * 2 * P) : 0;
  const int64_t pend = d > 0 ? round8(2 * (int64_t)(d + 1) * N * es) : 0;
  return round8((int64_t)(d + 2) * N * es) + round8(2 * N * es) + pend + table + kAdjWaves * 8;
}

// x - y wrapped into [0, m) for 0 <= x < m, 0 <= y < m.
__device__ __forceinline__ int wrap_sub(int x, int y, int m) { return x >= y ? x - y : x - y + m; }
// x + y wrapped into [0, m) for 0 <= x < m, 0 <= y < m.
__device__ __forceinline__ int wrap_add(int x, int y, int m) { return x + y >= m ? x + y - m : x + y; }

// kRing: the periodic ring (every point updated, neighbours wrap around, no
// end values); otherwise the Dirichlet rod (points 1..N-2).
template <typename F, int PPT, bool kRing>
__global__ __launch_bounds__(kAdjThreads) void ensemble_adjoint_kernel(EnsAdjDev a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int N = a.N, P = a.P, d = a.d, K = a.K;
  const int Q = d + 2;   // state slots and delay rows
  const int QP = d + 1;  // accumulator rows: landing steps k-d .. k
  F* uring = reinterpret_cast<F*>(smem);                       // state s in slot s % Q
  F* lring = reinterpret_cast<F*>(smem + a.uring_bytes);       // lambda(s) in row s % 2
  F* pend = reinterpret_cast<F*>(smem + a.uring_bytes + a.lring_bytes);
  // pend[(s % QP) * 2N + j]: delayed left reads of point j by point j+1 that
  // landed on step s; pend[(s % QP) * 2N + N + j]: delayed right reads of j by j-1
  uint8_t* dtab = smem + a.uring_bytes + a.lring_bytes + a.pend_bytes;  // step s: row s % Q
  double* wpart = reinterpret_cast<double*>(smem + a.uring_bytes + a.lring_bytes + a.pend_bytes +
                                            a.dtab_bytes);
  const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  const int64_t e = blockIdx.x;
  const uint64_t seed = a.seeds[e];
  const F* __restrict__ traj = static_cast<const F*>(a.traj) + e * (int64_t)(K + 1) * N;
  const F* __restrict__ gK = static_cast<const F*>(a.gK) + e * N;
  const F c1 = (F)a.c1, cN = (F)a.cN, r = (F)a.r;
  const int ndraw = d > 0 ? 2 * P : 0;
  const uint32_t dp1 = (uint32_t)d + 1;
  const int first = kRing ? 0 : 1, last = kRing ? N : N - 1;  // updated points [first, last)
  // the neighbours of point j, and whether they are updated points (readers)
  auto left_of = [&](int j) { return (kRing && j == 0) ? N - 1 : j - 1; };
  auto right_of = [&](int j) { return (kRing && j == N - 1) ? 0 : j + 1; };

  // my points j = first + tid + i*256: their own subdomain flags, those of
  // the neighbours that read them, and lambda_j(K) = gK_j
  int32_t mt[PPT], mtl[PPT], mtr[PPT];
  F lam[PPT];
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int j = first + tid + i * kAdjThreads;
    const bool ok = j < last;
    mt[i] = ok ? point_meta<kRing>(j, N, P) : 0;
    mtl[i] = ok && (kRing || j - 1 >= 1) ? point_meta<kRing>(left_of(j), N, P) : 0;
    mtr[i] = ok && (kRing || j + 1 <= N - 2) ? point_meta<kRing>(right_of(j), N, P) : 0;
    lam[i] = ok ? gK[j] : F(0);
    if (ok) lring[(K & 1) * N + j] = lam[i];
  }
  // Dirichlet: ends of every state slot, lambda 0 at the ends; accumulators start at 0
  if (!kRing) {
    for (int s = tid; s < Q; s += kAdjThreads) {
      uring[s * N] = c1;
      uring[s * N + N - 1] = cN;
    }
    if (tid < 2) {
      lring[tid * N] = 0;
      lring[tid * N + N - 1] = 0;
    }
  }
  if (ndraw)
    for (int q = tid; q < QP * 2 * N; q += kAdjThreads) pend[q] = F(0);
  // the states steps K-1 .. K-1-d read, and the delays of step K-1
  for (int s = K - 1; s >= 0 && s >= K - 1 - d; --s)
    for (int j = first + tid; j < last; j += kAdjThreads) uring[(s % Q) * N + j] = traj[(int64_t)s * N + j];
  if (K >= 1)
    for (int q = kAdjThreads - 1 - tid; q < ndraw; q += kAdjThreads)
      dtab[((K - 1) % Q) * ndraw + q] =
          (uint8_t)delay_at(seed, 2 * (uint64_t)(K - 1) * (uint64_t)P + (uint64_t)q, dp1);
  __syncthreads();

  double gr = 0.0, gc1 = 0.0, gcN = 0.0;
  int kq = K >= 1 ? (K - 1) % Q : 0;     // k % Q for the step k being reversed
  int kp = K >= 1 ? (K - 1) % QP : 0;    // k % QP
  // State k-d-1 enters the ring at step k (into the slot of state k+1, read
  // for the last time before the previous barrier).  It is loaded from HBM
  // four steps earlier into one of four register sets that the steps use in
  // turn, so the loads' latency hides behind four steps of work; every step
  // issues the same loads (clamped addresses), which keeps the wait counts
  // exact.
  auto load_state = [&](F (&pre)[PPT], int st) {
    const int64_t row = (int64_t)(st > 0 ? st : 0) * N;
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int j = first + tid + i * kAdjThreads;
      pre[i] = traj[row + (j < last ? j : last - 1)];
    }
  };
  auto step = [&](int k, F (&pre)[PPT]) {
    const int kq1 = wrap_add(kq, 1, Q);  // slot of k+1
    const int sp = k - d - 1;
    if (sp >= 0) {
      F* dst = uring + kq1 * N;  // (k-d-1) % Q == (k+1) % Q
#pragma unroll
      for (int i = 0; i < PPT; ++i) {
        const int j = first + tid + i * kAdjThreads;
        if (j < last) dst[j] = pre[i];
      }
    }
    load_state(pre, sp - 4);
    // the delays of step k-1, drawn by every thread
    if (k >= 1) {
      uint8_t* wrow = dtab + wrap_sub(kq, 1, Q) * ndraw;
      const uint64_t base = 2 * (uint64_t)(k - 1) * (uint64_t)P;
      for (int q = kAdjThreads - 1 - tid; q < ndraw; q += kAdjThreads)
        wrow[q] = (uint8_t)delay_at(seed, base + q, dp1);
    }
    const F* lam1 = lring + ((k + 1) & 1) * N;  // lambda(k+1)
    F* lam0 = lring + (k & 1) * N;              // lambda(k)
    const F* ucur = uring + kq * N;             // u(k)
    const uint8_t* drow = dtab + kq * ndraw;
    F* prow = pend + kp * 2 * N;                // accumulators of landing step k
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int j = first + tid + i * kAdjThreads;
      if (j < last) {
        const F lc = lam[i];
        const int jl = left_of(j), jr = right_of(j);
        // delays of this point's reads at step k, and of the neighbours' reads of it
        const bool eL = ndraw && (mt[i] & kEdgeLeft), eR = ndraw && (mt[i] & kEdgeRight);
        const bool nR = kRing || j + 1 <= N - 2, nL = kRing || j - 1 >= 1;  // updated neighbours
        const bool rEdge = ndraw && (mtr[i] & kEdgeLeft), lEdge = ndraw && (mtl[i] & kEdgeRight);
        const int pj = 2 * (mt[i] & 0x3fffffff);
        const int dl = eL ? drow[pj] : 0;
        const int dr = eR ? drow[pj + 1] : 0;
        const int dnr = rEdge ? drow[2 * (mtr[i] & 0x3fffffff)] : 0;
        const int dnl = lEdge ? drow[2 * (mtl[i] & 0x3fffffff) + 1] : 0;
        const int sL = k - dl > 0 ? k - dl : 0, sR = k - dr > 0 ? k - dr : 0;
        // dL/dr: the Laplacian term of this point's step
        const F uL = uring[wrap_sub(kq, k - sL, Q) * N + jl];
        const F uR = uring[wrap_sub(kq, k - sR, Q) * N + jr];
        const F lap = fma_of(F(-2), ucur[j], uL + uR);
        gr = __builtin_fma((double)lc, (double)lap, gr);
        if (!kRing && j == 1) gc1 = __builtin_fma((double)r, (double)lc, gc1);
        if (!kRing && j == N - 2) gcN = __builtin_fma((double)r, (double)lc, gcN);
        // reads of point j that landed on step k: direct ones now, delayed
        // ones from the accumulators (then cleared for landing step k-d-1)
        F nb = F(0);
        // (a read lands on its own step unless it is delayed and k > 0)
        if (nR && (!rEdge || dnr == 0 || k == 0)) nb += lam1[jr];
        if (nL && (!lEdge || dnl == 0 || k == 0)) nb += lam1[jl];
        if (ndraw) {
          nb += prow[j] + prow[N + j];
          prow[j] = F(0);
          prow[N + j] = F(0);
        }
        const F lnew = fma_of(r, fma_of(F(-2), lc, nb), lc);
        lam0[j] = lnew;
        lam[i] = lnew;
        // this point's delayed reads: add lambda_j(k+1) to the accumulator of
        // the step they landed on (nothing else writes those two entries now)
        if (nL && sL < k) {
          F* acc = pend + (wrap_sub(kp, k - sL, QP)) * 2 * N + jl;
          *acc += lc;
        }
        if (nR && sR < k) {
          F* acc = pend + (wrap_sub(kp, k - sR, QP)) * 2 * N + N + jr;
          *acc += lc;
        }
      }
    }
    __syncthreads();
    kq = wrap_sub(kq, 1, Q);
    kp = wrap_sub(kp, 1, QP);
  };
  F pre0[PPT], pre1[PPT], pre2[PPT], pre3[PPT];
  load_state(pre0, K - d - 2);
  load_state(pre1, K - d - 3);
  load_state(pre2, K - d - 4);
  load_state(pre3, K - d - 5);
  int k = K - 1;
  for (; k >= 3; k -= 4) {  // whole rounds of the four sets: no exit inside a round
    step(k, pre0);
    step(k - 1, pre1);
    step(k - 2, pre2);
    step(k - 3, pre3);
  }
  if (k >= 0) step(k--, pre0);
  if (k >= 0) step(k--, pre1);
  if (k >= 0) step(k--, pre2);

  // lambda(0)
  F* __restrict__ gu = static_cast<F*>(a.grad_u0) + e * N;
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int j = first + tid + i * kAdjThreads;
    if (j < last) gu[j] = lam[i];
  }
  if (kRing) {
    if (tid == 0) {  // the ring has no end values
      a.grad_c1[e] = 0.0;
      a.grad_cN[e] = 0.0;
    }
  } else {
    if (tid == 0) {
      gu[0] = F(0);
      gu[N - 1] = F(0);
      a.grad_c1[e] = gc1 + (double)gK[0];
    }
    if (((N - 2 - 1) % kAdjThreads) == tid) a.grad_cN[e] = gcN + (double)gK[N - 1];
  }
  gr = wave_sum_to_last(gr);
  if (lane == kWave - 1) wpart[wave] = gr;
  __syncthreads();
  if (tid == 0)
    a.grad_r[e] = ((wpart[0] + wpart[1]) + (wpart[2] + wpart[3])) +
                  ((wpart[4] + wpart[5]) + (wpart[6] + wpart[7]));
}

// Points per thread the kernel is built for.
static int ensemble_ppt(int64_t need) {
  for (int p : {1, 2, 4, 8, 12, 16})
    if (need <= p) return p;
  return 0;
}

template <typename F, bool kRing>
static hipError_t ensemble_dispatch(int ppt, dim3 grid, dim3 block, size_t lds, hipStream_t s,
                                    const EnsDev& a) {
  switch (ppt) {
    case 1: hipLaunchKernelGGL((ensemble_kernel<F, 1, kRing>), grid, block, lds, s, a); break;
    case 2: hipLaunchKernelGGL((ensemble_kernel<F, 2, kRing>), grid, block, lds, s, a); break;
    case 4: hipLaunchKernelGGL((ensemble_kernel<F, 4, kRing>), grid, block, lds, s, a); break;
    case 8: hipLaunchKernelGGL((ensemble_kernel<F, 8, kRing>), grid, block, lds, s, a); break;
    case 12: hipLaunchKernelGGL((ensemble_kernel<F, 12, kRing>), grid, block, lds, s, a); break;
    case 16: hipLaunchKernelGGL((ensemble_kernel<F, 16, kRing>), grid, block, lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ensemble(const EnsembleLaunch& L, hipStream_t s) {
  if (L.E < 1 || L.E > 0x7fffffffLL || L.N < 3 || L.P < 1 || L.P > L.N || L.K < 0 || L.d < 0 ||
      L.every < 1)
    return hipErrorInvalidValue;
  const int64_t lds = ensemble_lds_bytes(L.dtype, L.N, L.P, L.d);
  if (lds > kEnsembleMaxLds) return hipErrorInvalidValue;
  const int64_t es = L.dtype == 0 ? 4 : 8;
  const int64_t count = L.periodic ? L.N : L.N - 2;  // updated points
  const int ppt = ensemble_ppt((count + kFwdThreads - 1) / kFwdThreads);
  if (ppt == 0) return hipErrorInvalidValue;
  EnsDev a;
  a.u0 = L.u0;
  a.uK = L.uK;
  a.traj = L.traj;
  a.seeds = L.seeds;
  a.norms = L.norms;
  a.nobs = (int64_t)(L.K / L.every) + 1;
  a.N = L.N;
  a.P = L.P;
  a.K = L.K;
  a.d = L.d;
  a.Q = L.d + 2;
  a.every = L.every;
  a.ring_bytes = (int32_t)round8((int64_t)a.Q * L.N * es);
  a.dtab_bytes = L.d > 0 ? (int32_t)round8(4 * (int64_t)L.P) : 0;
  a.r = L.r;
  a.c1 = L.c1;
  a.cN = L.cN;
  if (L.nsnap < 0 || L.nsnap > kEnsembleMaxSnaps || (L.nsnap > 0 && !L.snaps))
    return hipErrorInvalidValue;
  a.snaps = L.nsnap > 0 ? L.snaps : nullptr;
  a.nsnap = L.nsnap;
  for (int j = 0; j < kEnsembleMaxSnaps; ++j) a.snap_steps[j] = j < L.nsnap ? L.snap_steps[j] : -1;
  const dim3 grid((unsigned)L.E), block((unsigned)kFwdThreads);
  const size_t sh = (size_t)lds;
  if (L.periodic)
    return L.dtype == 0 ? ensemble_dispatch<float, true>(ppt, grid, block, sh, s, a)
                        : ensemble_dispatch<double, true>(ppt, grid, block, sh, s, a);
  return L.dtype == 0 ? ensemble_dispatch<float, false>(ppt, grid, block, sh, s, a)
                      : ensemble_dispatch<double, false>(ppt, grid, block, sh, s, a);
}

template <typename F, bool kRing>
static hipError_t ensemble_adjoint_dispatch(int ppt, dim3 grid, size_t lds, hipStream_t s,
                                            const EnsAdjDev& a) {
  const dim3 block(kAdjThreads);
  switch (ppt) {
    case 1: hipLaunchKernelGGL((ensemble_adjoint_kernel<F, 1, kRing>), grid, block, lds, s, a); break;
    case 2: hipLaunchKernelGGL((ensemble_adjoint_kernel<F, 2, kRing>), grid, block, lds, s, a); break;
    case 4: hipLaunchKernelGGL((ensemble_adjoint_kernel<F, 4, kRing>), grid, block, lds, s, a); break;
    case 8: hipLaunchKernelGGL((ensemble_adjoint_kernel<F, 8, kRing>), grid, block, lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ensemble_adjoint(const EnsembleAdjointLaunch& L, hipStream_t s) {
  if (L.E < 1 || L.E > 0x7fffffffLL || L.N < 3 || L.P < 1 || L.P > L.N || L.K < 0 || L.d < 0 ||
      !L.traj || !L.gK || !L.seeds || !L.grad_u0 || !L.grad_r || !L.grad_c1 || !L.grad_cN)
    return hipErrorInvalidValue;
  const int64_t lds = ensemble_adjoint_lds_bytes(L.dtype, L.N, L.P, L.d);
  if (lds > kEnsembleMaxLds) return hipErrorInvalidValue;
  const int64_t count = L.periodic ? L.N : L.N - 2;  // updated points
  const int ppt = ensemble_ppt((count + kAdjThreads - 1) / kAdjThreads);
  if (ppt == 0 || ppt > 8) return hipErrorInvalidValue;
  const int64_t es = L.dtype == 0 ? 4 : 8;
  EnsAdjDev a;
  a.traj = L.traj;
  a.gK = L.gK;
  a.seeds = L.seeds;
  a.grad_u0 = L.grad_u0;
  a.grad_r = L.grad_r;
  a.grad_c1 = L.grad_c1;
  a.grad_cN = L.grad_cN;
  a.N = L.N;
  a.P = L.P;
  a.K = L.K;
  a.d = L.d;
  a.uring_bytes = (int32_t)round8((int64_t)(L.d + 2) * L.N * es);
  a.lring_bytes = (int32_t)round8(2 * (int64_t)L.N * es);
  a.pend_bytes = L.d > 0 ? (int32_t)round8(2 * (int64_t)(L.d + 1) * L.N * es) : 0;
  a.dtab_bytes = L.d > 0 ? (int32_t)round8((int64_t)(L.d + 2) * 2 * L.P) : 0;
  a.r = L.r;
  a.c1 = L.c1;
  a.cN = L.cN;
  const dim3 grid((unsigned)L.E);
  if (L.periodic)
    return L.dtype == 0 ? ensemble_adjoint_dispatch<float, true>(ppt, grid, (size_t)lds, s, a)
                        : ensemble_adjoint_dispatch<double, true>(ppt, grid, (size_t)lds, s, a);
  return L.dtype == 0 ? ensemble_adjoint_dispatch<float, false>(ppt, grid, (size_t)lds, s, a)
                      : ensemble_adjoint_dispatch<double, false>(ppt, grid, (size_t)lds, s, a);
}

}  // namespace heat1d
