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
// Steps are HBM-bound: a forward step reads and writes the state (2 s bytes
// per point), a backward step reads lambda(k+1) and u(k) and writes lambda(k)
// (3 s bytes per point); the edge records add 2 values per edge and step.
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

__global__ void partition_kernel(int64_t* __restrict__ lo, int64_t N, int P) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p <= P) lo[p] = (int64_t)p * N / P;
}

// E[k][b] for every edge b from the state u(k).
template <typename F>
__global__ void edges_from_state_kernel(const F* __restrict__ u, F* __restrict__ Ek,
                                        const int64_t* __restrict__ lo, int P) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < 1 || b >= P) return;
  Ek[2 * b] = u[lo[b] - 1];
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
  __device__ __forceinline__ bool first(int64_t i) const { return p > 0 && i == lo_p; }
  __device__ __forceinline__ bool last(int64_t i, int P) const {
    return p + 1 < P && i == lo_p1 - 1;
  }
};

__device__ __forceinline__ EdgeScan edge_scan(int64_t i0, const int64_t* __restrict__ lo, int P,
                                              double pscale) {
  EdgeScan e;
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
template <typename F>
__global__ __launch_bounds__(kThreads) void async_lockstep_kernel(
    const F* __restrict__ cur, F* __restrict__ nxt, F* __restrict__ E,
    const int64_t* __restrict__ lo, int64_t N, int P, int k, int d, uint64_t seed, F r, F c1,
    F cN, double pscale, int record, int aligned) {
  const int64_t i0 = ((int64_t)blockIdx.x * kThreads + threadIdx.x) * kPts;
  if (i0 >= N) return;
  F c[kPts], v[kPts];
  load_points<F, kPts>(c, cur, i0, N, aligned != 0);
  const F before = i0 >= 1 ? cur[i0 - 1] : F(0);
  const F after = i0 + kPts < N ? cur[i0 + kPts] : F(0);
  EdgeScan es = edge_scan(i0, lo, P, pscale);
  const bool plain = !(es.p + 1 < P && es.lo_p1 - 1 <= i0 + kPts - 1) &&
                     !(es.p > 0 && es.lo_p == i0) && i0 >= 1 && i0 + kPts <= N - 1;
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
      if (i == 0) {
        val = c1;
      } else if (i == N - 1) {
        val = cN;
      } else {
        F left = j > 0 ? c[j - 1] : before, right = j + 1 < kPts ? c[j + 1] : after;
        if (first) {
          const int dl = delay_of(seed, k, es.p, 0, P, d);
          left = E[((int64_t)(k - dl > 0 ? k - dl : 0) * P + es.p) * 2];
        }
        if (last) {
          const int dr = delay_of(seed, k, es.p, 1, P, d);
          right = E[((int64_t)(k - dr > 0 ? k - dr : 0) * P + es.p + 1) * 2 + 1];
        }
        val = eq3_step(left, c[j], right, r);
      }
      v[j] = val;
      if (record) {
        if (first) E[((int64_t)(k + 1) * P + es.p) * 2 + 1] = val;
        if (last) E[((int64_t)(k + 1) * P + es.p + 1) * 2] = val;
      }
    }
  }
  store_points<F, kPts>(v, nxt, i0, 0, 0, (int)(N - i0 < kPts ? N - i0 : kPts), aligned != 0);
}

// lambda(k) from lambda(k+1) and u(k) (the transpose of the step above), the
// dL/dr term of step k summed per workgroup into part[blockIdx.x], and the
// dL/dc1, dL/dcN terms of step k added to ends[0], ends[1].  Each workgroup
// owns its partial slot and the grid is the same for every step, so the sums
// run in a fixed order.
template <typename F>
__global__ __launch_bounds__(kThreads) void async_adjoint_step_kernel(
    const F* __restrict__ lam1, F* __restrict__ lam0, const F* __restrict__ u,
    const F* __restrict__ E, F* __restrict__ LE, const int64_t* __restrict__ lo, int64_t N,
    int P, int k, int K, int d, uint64_t seed, F r, double pscale, double* __restrict__ part,
    double* __restrict__ ends, int aligned) {
  __shared__ double red[kThreads / kWave];
  const int64_t i0 = ((int64_t)blockIdx.x * kThreads + threadIdx.x) * kPts;
  double g = 0.0;
  if (i0 < N) {
    F l[kPts], c[kPts], out[kPts];
    load_points<F, kPts>(l, lam1, i0, N, aligned != 0);
    load_points<F, kPts>(c, u, i0, N, aligned != 0);
    const F lb = i0 >= 1 ? lam1[i0 - 1] : F(0), la = i0 + kPts < N ? lam1[i0 + kPts] : F(0);
    const F ub = i0 >= 1 ? u[i0 - 1] : F(0), ua = i0 + kPts < N ? u[i0 + kPts] : F(0);
    EdgeScan es = edge_scan(i0, lo, P, pscale);
    const bool plain = !(es.p + 1 < P && es.lo_p1 - 1 <= i0 + kPts - 1) &&
                       !(es.p > 0 && es.lo_p == i0) && i0 >= 2 && i0 + kPts <= N - 2;
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
        if (i < 1 || i > N - 2) continue;
        es.to(i, lo, P);
        const int p = es.p;
        const bool first = es.first(i), last = es.last(i, P);
        const F l1 = l[j];
        // dL/dr: lambda_i(k+1) times the Laplacian the forward step used
        F uL = j > 0 ? c[j - 1] : ub, uR = j + 1 < kPts ? c[j + 1] : ua;
        if (first) {
          const int dl = delay_of(seed, k, p, 0, P, d);
          uL = E[((int64_t)(k - dl > 0 ? k - dl : 0) * P + p) * 2];
        }
        if (last) {
          const int dr = delay_of(seed, k, p, 1, P, d);
          uR = E[((int64_t)(k - dr > 0 ? k - dr : 0) * P + p + 1) * 2 + 1];
        }
        g += (double)l1 * ((double)uL + (double)uR - 2.0 * (double)c[j]);
        // the neighbours' reads of u_i(k)
        F nb = F(0);
        if (i + 1 <= N - 2) {
          if (last) {  // point i+1 opens subdomain p+1 and read u_i with its left delays
            for (int kk = k; kk <= kmax; ++kk) {
              const int dl = delay_of(seed, kk, p + 1, 0, P, d);
              if ((kk - dl > 0 ? kk - dl : 0) == k)
                nb += LE[((int64_t)(kk + 1) * P + p + 1) * 2 + 1];
            }
          } else {
            nb += j + 1 < kPts ? l[j + 1] : la;
          }
        }
        if (i - 1 >= 1) {
          if (first) {  // point i-1 closes subdomain p-1 and read u_i with its right delays
            for (int kk = k; kk <= kmax; ++kk) {
              const int dr = delay_of(seed, kk, p - 1, 1, P, d);
              if ((kk - dr > 0 ? kk - dr : 0) == k) nb += LE[((int64_t)(kk + 1) * P + p) * 2];
            }
          } else {
            nb += j > 0 ? l[j - 1] : lb;
          }
        }
        const F lnew = fma_of(r, fma_of(F(-2), l1, nb), l1);
        out[j] = lnew;
        if (first) LE[((int64_t)k * P + p) * 2 + 1] = lnew;
        if (last) LE[((int64_t)k * P + p + 1) * 2] = lnew;
        if (i == 1) ends[0] += (double)r * (double)l1;
        if (i == N - 2) ends[1] += (double)r * (double)l1;
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
                                    double* grad_cN) {
  if (threadIdx.x == 0) {
    *grad_c1 = (double)gK[0] + ends[0];
    *grad_cN = (double)gK[N - 1] + ends[1];
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
                              hipStream_t s) {
  if (P < 2) return hipSuccess;
  const dim3 grid((unsigned)((P + 255) / 256));
  if (dtype == 0)
    hipLaunchKernelGGL(edges_from_state_kernel<float>, grid, dim3(256), 0, s, (const float*)u,
                       (float*)Ek, lo, P);
  else
    hipLaunchKernelGGL(edges_from_state_kernel<double>, grid, dim3(256), 0, s, (const double*)u,
                       (double*)Ek, lo, P);
  return hipGetLastError();
}

hipError_t launch_async_lockstep(const AsyncAdjStep& a, const void* cur, void* nxt, int k,
                                 int record, hipStream_t s) {
  const dim3 grid((unsigned)async_adjoint_blocks(a.N));
  const double pscale = (double)a.P / (double)a.N;
  if (a.dtype == 0)
    hipLaunchKernelGGL(async_lockstep_kernel<float>, grid, dim3(kThreads), 0, s,
                       (const float*)cur, (float*)nxt, (float*)a.E, a.lo, a.N, a.P, k, a.d,
                       a.seed, (float)a.r, (float)a.c1, (float)a.cN, pscale, record,
                       aligned_pair(cur, nxt, a.N));
  else
    hipLaunchKernelGGL(async_lockstep_kernel<double>, grid, dim3(kThreads), 0, s,
                       (const double*)cur, (double*)nxt, (double*)a.E, a.lo, a.N, a.P, k, a.d,
                       a.seed, a.r, a.c1, a.cN, pscale, record, aligned_pair(cur, nxt, a.N));
  return hipGetLastError();
}

hipError_t launch_async_adjoint_step(const AsyncAdjStep& a, const void* lam1, void* lam0,
                                     const void* u, int k, hipStream_t s) {
  const dim3 grid((unsigned)async_adjoint_blocks(a.N));
  const double pscale = (double)a.P / (double)a.N;
  if (a.dtype == 0)
    hipLaunchKernelGGL(async_adjoint_step_kernel<float>, grid, dim3(kThreads), 0, s,
                       (const float*)lam1, (float*)lam0, (const float*)u, (const float*)a.E,
                       (float*)a.LE, a.lo, a.N, a.P, k, a.K, a.d, a.seed, (float)a.r, pscale,
                       a.part, a.ends, aligned_pair(lam1, lam0, a.N) && is_aligned16(u));
  else
    hipLaunchKernelGGL(async_adjoint_step_kernel<double>, grid, dim3(kThreads), 0, s,
                       (const double*)lam1, (double*)lam0, (const double*)u, (const double*)a.E,
                       (double*)a.LE, a.lo, a.N, a.P, k, a.K, a.d, a.seed, a.r, pscale, a.part,
                       a.ends, aligned_pair(lam1, lam0, a.N) && is_aligned16(u));
  return hipGetLastError();
}

hipError_t launch_async_adjoint_ends(int dtype, const void* gK, int64_t N, const double* ends,
                                     double* grad_c1, double* grad_cN, hipStream_t s) {
  if (dtype == 0)
    hipLaunchKernelGGL(adjoint_ends_kernel<float>, dim3(1), dim3(64), 0, s, (const float*)gK, N,
                       ends, grad_c1, grad_cN);
  else
    hipLaunchKernelGGL(adjoint_ends_kernel<double>, dim3(1), dim3(64), 0, s, (const double*)gK,
                       N, ends, grad_c1, grad_cN);
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
