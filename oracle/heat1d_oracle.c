/*
 * heat1d_oracle.c -- plain FP64 CPU reference for the 1D heat-equation hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it (through oracle/__init__.py).  It shares no code, no
 * header and no table with the GPU path.
 *
 * Everything here is written for clarity, not speed: two full buffers per step,
 * index-order loops, no blocking and no fusion.  It is compiled with
 * -ffp-contract=off so every product and sum is rounded separately, exactly as
 * the printed formulas read.  The only concession to size is an OpenMP pragma on
 * the independent spatial loop of one time step (and on the independent rods of
 * a batch), which does not change any result.
 *
 * Indexing: 0-based.  The paper numbers the grid points 1..N; its point i is
 * our point i-1, so the two Dirichlet ends are points 0 and N-1.
 *
 * Paper: K. Lee and R. Bhattacharya, "Asynchronous Parallel Computing
 * Algorithm implemented in 1D Heat Equation with CUDA", arXiv:1510.08982.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL 1
#define ORACLE_ENOMEM 2

/* ------------------------------------------------------------------------- */
/* Eq.3 (Section 2): u_i(k+1) = r u_{i+1}(k) + (1-2r) u_i(k) + r u_{i-1}(k).   */
/* Evaluated left to right exactly as printed; w = 1-2r is formed once.         */
/* ------------------------------------------------------------------------- */
static double eq3(double u_right, double u_centre, double u_left, double r, double w)
{
    return r * u_right + w * u_centre + r * u_left;
}

/* Section 2: the stability range quoted for r is (0, 0.5]; the experiments of
 * Section 5 use the end point r = 0.5 itself. */
static int r_is_valid(double r) { return r > 0.0 && r <= 0.5; }

/*
 * Synchronous iteration of Eq.3 with the Dirichlet ends of Section 2
 * (u_1(k) = c1, u_N(k) = c2 for all k; c2 is called cN here).
 *
 * Works on a contiguous segment of a rod: the segment holds the global points
 * [gofs, gofs+len) of a rod of N points.  For the whole rod pass gofs = 0 and
 * len = N.  A segment end that is not a rod end has no neighbour outside the
 * segment, so that point is left at its input value; the result is then exact
 * only at distance >= K from such an end (the stencil spreads information by one
 * point per step), which is how a caller samples single outputs of a large rod.
 *
 * u_in and u_out hold len values and may not overlap.  The two Dirichlet
 * values overwrite whatever u_in holds at global points 0 and N-1, at k = 0 and
 * at every later step.
 */
int oracle_sync(int64_t len, int64_t gofs, int64_t N, const double *u_in,
                double r, double c1, double cN, int64_t K, double *u_out)
{
    if (len < 1 || N < 3 || gofs < 0 || gofs + len > N || K < 0 || !r_is_valid(r))
        return ORACLE_EINVAL;
    double *cur = (double *)malloc((size_t)len * sizeof(double));
    double *nxt = (double *)malloc((size_t)len * sizeof(double));
    if (!cur || !nxt) { free(cur); free(nxt); return ORACLE_ENOMEM; }

    const double w = 1.0 - 2.0 * r;
    memcpy(cur, u_in, (size_t)len * sizeof(double));
    if (gofs == 0) cur[0] = c1;
    if (gofs + len == N) cur[len - 1] = cN;

    for (int64_t k = 0; k < K; ++k) {
        /* both segment ends (Dirichlet ends or frozen cut points) keep their value */
        nxt[0] = cur[0];
        nxt[len - 1] = cur[len - 1];
#pragma omp parallel for schedule(static) if (len > 200000)
        for (int64_t i = 1; i < len - 1; ++i)
            nxt[i] = eq3(cur[i + 1], cur[i], cur[i - 1], r, w);
        double *t = cur; cur = nxt; nxt = t;
    }
    memcpy(u_out, cur, (size_t)len * sizeof(double));
    free(cur);
    free(nxt);
    return ORACLE_OK;
}

/* Batch of independent rods packed back to back: rod b holds the points
 * [offsets[b], offsets[b+1]) of u_in / u_out and has its own r, c1, cN, K. */
int oracle_sync_batched(int64_t nrods, const int64_t *offsets, const double *u_in,
                        const double *r, const double *c1, const double *cN,
                        const int64_t *K, double *u_out)
{
    int status = ORACLE_OK;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < nrods; ++b) {
        int64_t n = offsets[b + 1] - offsets[b];
        int s = oracle_sync(n, 0, n, u_in + offsets[b], r[b], c1[b], cN[b], K[b],
                            u_out + offsets[b]);
        if (s != ORACLE_OK) {
#pragma omp critical
            status = s;
        }
    }
    return status;
}

/* ------------------------------------------------------------------------- */
/* Delay schedule for the emulated asynchronous iteration.                      */
/*                                                                              */
/* Eq.4 only says each delayed read comes from one of the last q steps; the     */
/* schedule that picks the delay is ours.  It is a counter-based hash so that   */
/* any (step, subdomain, side) can be evaluated on its own.  The mixing         */
/* function is the output function of SplitMix64 (Steele, Lea and Flood,        */
/* "Fast splittable pseudorandom number generators", OOPSLA 2014): the state    */
/* advances by the 64-bit golden-ratio increment and the result is passed       */
/* through two xor-shift-multiply rounds and a final xor-shift.                 */
/*                                                                              */
/*   c     = ((k * P + p) << 1) | side            (side 0: left edge, 1: right) */
/*   x     = sm64(seed XOR sm64(c))                                             */
/*   delta = ((x >> 32) * (d + 1)) >> 32          (a value in 0..d)             */
/* ------------------------------------------------------------------------- */
uint64_t oracle_splitmix64(uint64_t state)
{
    uint64_t z = state + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int oracle_delay(uint64_t seed, int64_t k, int64_t p, int side, int64_t P, int d)
{
    uint64_t c = ((((uint64_t)k) * (uint64_t)P + (uint64_t)p) << 1) | (uint64_t)(side & 1);
    uint64_t x = oracle_splitmix64(seed ^ oracle_splitmix64(c));
    return (int)(((x >> 32) * (uint64_t)(d + 1)) >> 32);
}

/* out[(k*P + p)*2 + side] = delay, for k < K, p < P, side < 2. */
void oracle_delay_schedule(uint64_t seed, int64_t P, int64_t K, int d, uint8_t *out)
{
    for (int64_t k = 0; k < K; ++k)
        for (int64_t p = 0; p < P; ++p)
            for (int side = 0; side < 2; ++side)
                out[(k * P + p) * 2 + side] = (uint8_t)oracle_delay(seed, k, p, side, P, d);
}

/* Two fixed schedules beside the seeded one, for adversarial runs: kind 1 reads
 * every subdomain edge at the largest delay d (the oldest value Eq.4 allows),
 * kind 2 alternates between the newest and the oldest value step by step
 * (delay d on odd steps, 0 on even ones).  Kind 0 is the seeded draw above. */
int oracle_sched_delay(int kind, uint64_t seed, int64_t k, int64_t p, int side, int64_t P, int d)
{
    if (kind == 1) return d;
    if (kind == 2) return (k & 1) ? d : 0;
    return oracle_delay(seed, k, p, side, P, d);
}

/* Subdomain partition (Section 2, Fig. 1: a PE owns a group of grid points):
 * subdomain p owns [lo(p), lo(p+1)) with lo(p) = floor(p N / P). */
static int64_t sub_lo(int64_t p, int64_t N, int64_t P) { return (p * N) / P; }

/*
 * Emulated asynchronous iteration, Eq.4 (Section 3).
 *
 * The rod is split into P subdomains.  Inside a subdomain every neighbour read
 * is current (Section 3: no asynchrony inside a PE).  The first point of
 * subdomain p > 0 reads its left neighbour (the last point of p-1) at step
 * max(0, k - delta(k, p, 0)); the last point of subdomain p < P-1 reads its
 * right neighbour (the first point of p+1) at step max(0, k - delta(k, p, 1)).
 * Delays lie in 0..d, so the read step lies in {k, ..., k-q+1} with q = d+1,
 * the buffer length of Eq.4.  Steps before 0 are read as step 0 (the initial
 * state with its Dirichlet ends).
 *
 * The oracle simply keeps the last d+2 whole states in a ring (the d+1 states
 * a read may use plus the one being written).  As in
 * oracle_sync, (u_in, u_out) may be a segment [gofs, gofs+len) of the rod; the
 * subdomain partition is always that of the whole rod of N points.
 */
/* Euclidean norm of a state, the squares summed in index order (Section 5,
 * Fig. 3 plots this 2-norm of the whole state u(k), ends included). */
static double state_norm(int64_t len, const double *u)
{
    double acc = 0.0;
    for (int64_t i = 0; i < len; ++i) acc += u[i] * u[i];
    return sqrt(acc);
}

/* The iteration itself; when norms != NULL it also stores the norm of u(j*every)
 * in norms[j] for j = 0 .. K/every. */
static int async_run(int64_t len, int64_t gofs, int64_t N, int64_t P,
                     const double *u_in, double r, double c1, double cN,
                     int64_t K, int d, uint64_t seed, int kind, double *u_out,
                     int64_t every, double *norms)
{
    if (len < 1 || N < 3 || gofs < 0 || gofs + len > N || K < 0 || !r_is_valid(r) ||
        d < 0 || P < 1 || P > N || kind < 0 || kind > 2)
        return ORACLE_EINVAL;
    const int64_t Q = (int64_t)d + 2;
    double *hist = (double *)malloc((size_t)(Q * len) * sizeof(double));
    int64_t *sub = (int64_t *)malloc((size_t)len * sizeof(int64_t));
    signed char *edge = (signed char *)malloc((size_t)len);
    if (!hist || !sub || !edge) { free(hist); free(sub); free(edge); return ORACLE_ENOMEM; }

    /* which subdomain each point belongs to, and whether it is a left (bit 0)
     * or right (bit 1) subdomain edge with a neighbour subdomain */
    {
        int64_t p = 0;
        while (p + 1 < P && sub_lo(p + 1, N, P) <= gofs) ++p;
        for (int64_t i = 0; i < len; ++i) {
            int64_t g = gofs + i;
            while (p + 1 < P && sub_lo(p + 1, N, P) <= g) ++p;
            sub[i] = p;
            edge[i] = 0;
            if (p > 0 && g == sub_lo(p, N, P)) edge[i] |= 1;
            if (p < P - 1 && g == sub_lo(p + 1, N, P) - 1) edge[i] |= 2;
        }
    }

    const double w = 1.0 - 2.0 * r;
    double *u0 = hist; /* slot 0 holds step 0 */
    memcpy(u0, u_in, (size_t)len * sizeof(double));
    if (gofs == 0) u0[0] = c1;
    if (gofs + len == N) u0[len - 1] = cN;
    if (norms) norms[0] = state_norm(len, u0);

    for (int64_t k = 0; k < K; ++k) {
        const double *cur = hist + (k % Q) * len;
        double *nxt = hist + ((k + 1) % Q) * len;
        nxt[0] = cur[0];
        nxt[len - 1] = cur[len - 1];
#pragma omp parallel for schedule(static) if (len > 200000)
        for (int64_t i = 1; i < len - 1; ++i) {
            double left = cur[i - 1];
            double right = cur[i + 1];
            if (edge[i] & 1) {
                int64_t ks = k - oracle_sched_delay(kind, seed, k, sub[i], 0, P, d);
                if (ks < 0) ks = 0;
                left = hist[(ks % Q) * len + (i - 1)];
            }
            if (edge[i] & 2) {
                int64_t ks = k - oracle_sched_delay(kind, seed, k, sub[i], 1, P, d);
                if (ks < 0) ks = 0;
                right = hist[(ks % Q) * len + (i + 1)];
            }
            nxt[i] = eq3(right, cur[i], left, r, w);
        }
        if (norms && (k + 1) % every == 0) norms[(k + 1) / every] = state_norm(len, nxt);
    }
    memcpy(u_out, hist + (K % Q) * len, (size_t)len * sizeof(double));
    free(hist);
    free(sub);
    free(edge);
    return ORACLE_OK;
}

int oracle_async_emulated(int64_t len, int64_t gofs, int64_t N, int64_t P,
                          const double *u_in, double r, double c1, double cN,
                          int64_t K, int d, uint64_t seed, double *u_out)
{
    return async_run(len, gofs, N, P, u_in, r, c1, cN, K, d, seed, 0, u_out, 1, NULL);
}

/* The same run under schedule `kind` (0 seeded, 1 every read at delay d,
 * 2 delay d on odd steps and 0 on even ones). */
int oracle_async_emulated_kind(int64_t len, int64_t gofs, int64_t N, int64_t P,
                               const double *u_in, double r, double c1, double cN,
                               int64_t K, int d, uint64_t seed, int kind, double *u_out)
{
    return async_run(len, gofs, N, P, u_in, r, c1, cN, K, d, seed, kind, u_out, 1, NULL);
}

/*
 * The same emulated iteration with the periodic boundary of Section 5.3: the
 * two end points are neighbours of each other, so every point of the ring of N
 * points takes the Eq.3 update, point 0 reading point N-1 as its left
 * neighbour and point N-1 reading point 0 as its right one (two buffers, as
 * for the Dirichlet rod).  With P > 1 subdomains every subdomain has both
 * edges: the first point of subdomain 0 reads the last point of subdomain P-1
 * with the delay of (k, 0, left), and the last point of subdomain P-1 reads
 * point 0 with the delay of (k, P-1, right).  With P = 1 nothing is delayed.
 */
static int async_run_periodic(int64_t N, int64_t P, const double *u_in, double r, int64_t K,
                              int d, uint64_t seed, double *u_out, int64_t every,
                              double *norms)
{
    if (N < 3 || K < 0 || !r_is_valid(r) || d < 0 || P < 1 || P > N) return ORACLE_EINVAL;
    const int64_t Q = (int64_t)d + 2;
    double *hist = (double *)malloc((size_t)(Q * N) * sizeof(double));
    int64_t *sub = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    signed char *edge = (signed char *)malloc((size_t)N);
    if (!hist || !sub || !edge) { free(hist); free(sub); free(edge); return ORACLE_ENOMEM; }
    {
        int64_t p = 0;
        for (int64_t i = 0; i < N; ++i) {
            while (p + 1 < P && sub_lo(p + 1, N, P) <= i) ++p;
            sub[i] = p;
            edge[i] = 0;
            if (P > 1 && i == sub_lo(p, N, P)) edge[i] |= 1;
            if (P > 1 && i == sub_lo(p + 1, N, P) - 1) edge[i] |= 2;
        }
    }
    const double w = 1.0 - 2.0 * r;
    memcpy(hist, u_in, (size_t)N * sizeof(double));
    if (norms) norms[0] = state_norm(N, hist);
    for (int64_t k = 0; k < K; ++k) {
        const double *cur = hist + (k % Q) * N;
        double *nxt = hist + ((k + 1) % Q) * N;
        for (int64_t i = 0; i < N; ++i) {
            const int64_t il = (i == 0) ? N - 1 : i - 1;
            const int64_t ir = (i == N - 1) ? 0 : i + 1;
            double left = cur[il];
            double right = cur[ir];
            if (edge[i] & 1) {
                int64_t ks = k - oracle_delay(seed, k, sub[i], 0, P, d);
                if (ks < 0) ks = 0;
                left = hist[(ks % Q) * N + il];
            }
            if (edge[i] & 2) {
                int64_t ks = k - oracle_delay(seed, k, sub[i], 1, P, d);
                if (ks < 0) ks = 0;
                right = hist[(ks % Q) * N + ir];
            }
            nxt[i] = eq3(right, cur[i], left, r, w);
        }
        if (norms && (k + 1) % every == 0) norms[(k + 1) / every] = state_norm(N, nxt);
    }
    memcpy(u_out, hist + (K % Q) * N, (size_t)N * sizeof(double));
    free(hist);
    free(sub);
    free(edge);
    return ORACLE_OK;
}

/*
 * An ensemble of emulated asynchronous runs (Section 5, Fig. 3: many runs of
 * the same rod whose trajectories differ only through the random delays).
 * Member e starts from u_in + e*N, draws its delays with seeds[e] and ends in
 * u_out + e*N; norms + e*(K/every + 1) receives the 2-norm of its whole state
 * at steps 0, every, 2*every, ..., (K/every)*every.  Each member is exactly
 * oracle_async_emulated on its own (or, with periodic != 0, the periodic
 * iteration above, c1 and cN unused); members run in parallel.
 */
int oracle_async_ensemble(int64_t E, int64_t N, int64_t P, const double *u_in, double r,
                          double c1, double cN, int64_t K, int d, const uint64_t *seeds,
                          int64_t every, int periodic, double *u_out, double *norms)
{
    if (E < 1 || every < 1) return ORACLE_EINVAL;
    const int64_t nobs = K / every + 1;
    int status = ORACLE_OK;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t e = 0; e < E; ++e) {
        int st = periodic
                     ? async_run_periodic(N, P, u_in + e * N, r, K, d, seeds[e], u_out + e * N,
                                          every, norms + e * nobs)
                     : async_run(N, 0, N, P, u_in + e * N, r, c1, cN, K, d, seeds[e], 0,
                                 u_out + e * N, every, norms + e * nobs);
        if (st != ORACLE_OK) {
#pragma omp critical
            status = st;
        }
    }
    return status;
}

/* ------------------------------------------------------------------------- */
/* Discrete adjoint of the synchronous iteration (derived from Eq.3).          */
/*                                                                              */
/* For a loss L(u(K)) with gradient g = dL/du(K):                               */
/*   lambda(K) = g with both ends set to 0 (u(K) is fixed at the ends);          */
/*   for k = K-1 down to 0:                                                      */
/*     dL/dr += sum_{i=1}^{N-2} lambda_i(k+1) (u_{i+1}(k) - 2 u_i(k) + u_{i-1}(k)) */
/*     lambda_i(k) = r lambda_{i+1}(k+1) + (1-2r) lambda_i(k+1)                  */
/*                   + r lambda_{i-1}(k+1)     for i = 1..N-2, ends 0.            */
/*   dL/du0 = lambda(0) (its ends are 0: u0's ends are overwritten by c1, cN).   */
/*   dL/dc1 = gK[0] + r sum_{k=1..K} lambda_1(k), dL/dcN likewise with point     */
/*   N-2 (the ends hold c1, cN at every step and only points 1, N-2 read them).  */
/* The interior block of the Eq.3 matrix is symmetric, so its transpose is the  */
/* same stencil with homogeneous (zero) ends.                                   */
/*                                                                              */
/* The states u(k) are needed in reverse order.  If the whole trajectory fits   */
/* in 'full_traj_bytes' it is stored; otherwise every 64th state is kept and    */
/* the states of each 64-step stretch are recomputed from it when the backward   */
/* sweep reaches that stretch.                                                  */
/* ------------------------------------------------------------------------- */
static void sync_step_full(int64_t N, const double *cur, double *nxt, double r, double w)
{
    nxt[0] = cur[0];
    nxt[N - 1] = cur[N - 1];
#pragma omp parallel for schedule(static) if (N > 200000)
    for (int64_t i = 1; i < N - 1; ++i)
        nxt[i] = eq3(cur[i + 1], cur[i], cur[i - 1], r, w);
}

int oracle_adjoint(int64_t N, const double *u0, const double *gK, double r, double c1,
                   double cN, int64_t K, double *grad_u0, double *grad_r,
                   double *grad_c1, double *grad_cN, int64_t full_traj_bytes)
{
    if (N < 3 || K < 0 || !r_is_valid(r)) return ORACLE_EINVAL;
    const double w = 1.0 - 2.0 * r;
    const int64_t stride = 64;
    const int store_all = (double)(K + 1) * (double)N * 8.0 <= (double)full_traj_bytes;
    const int64_t nstates = store_all ? (K + 1) : (K / stride + 1);
    const int64_t nseg = store_all ? 0 : (stride + 1);
    double *traj = (double *)malloc((size_t)(nstates * N) * sizeof(double));
    double *seg = nseg ? (double *)malloc((size_t)(nseg * N) * sizeof(double)) : NULL;
    double *lam = (double *)malloc((size_t)N * sizeof(double));
    double *lam2 = (double *)malloc((size_t)N * sizeof(double));
    if (!traj || (nseg && !seg) || !lam || !lam2) {
        free(traj); free(seg); free(lam); free(lam2);
        return ORACLE_ENOMEM;
    }

    /* forward sweep: u(0) with its ends imposed, then Eq.3 */
    memcpy(traj, u0, (size_t)N * sizeof(double));
    traj[0] = c1;
    traj[N - 1] = cN;
    if (store_all) {
        for (int64_t k = 0; k < K; ++k)
            sync_step_full(N, traj + k * N, traj + (k + 1) * N, r, w);
    } else {
        double *a = lam, *b = lam2; /* borrowed as scratch before the backward sweep */
        memcpy(a, traj, (size_t)N * sizeof(double));
        for (int64_t k = 0; k < K; ++k) {
            sync_step_full(N, a, b, r, w);
            double *t = a; a = b; b = t;
            if ((k + 1) % stride == 0) memcpy(traj + ((k + 1) / stride) * N, a, (size_t)N * sizeof(double));
        }
    }

    /* backward sweep */
    for (int64_t i = 0; i < N; ++i) lam[i] = gK[i];
    lam[0] = 0.0;
    lam[N - 1] = 0.0;
    double gr = 0.0;
    /* u_0(k) = c1 for every k: point 1 reads it at every step with weight r,
     * and u_0(K) itself carries gK[0]; likewise cN through point N-2 */
    double gc1 = gK[0], gcN = gK[N - 1];
    int64_t seg_base = -1; /* first step held in seg[] */
    for (int64_t k = K - 1; k >= 0; --k) {
        const double *uk;
        if (store_all) {
            uk = traj + k * N;
        } else {
            int64_t base = (k / stride) * stride;
            if (base != seg_base) {
                memcpy(seg, traj + (base / stride) * N, (size_t)N * sizeof(double));
                for (int64_t j = 1; j < stride && base + j < K; ++j)
                    sync_step_full(N, seg + (j - 1) * N, seg + j * N, r, w);
                seg_base = base;
            }
            uk = seg + (k - base) * N;
        }
        for (int64_t i = 1; i < N - 1; ++i)
            gr += lam[i] * (uk[i + 1] - 2.0 * uk[i] + uk[i - 1]);
        gc1 += r * lam[1];
        gcN += r * lam[N - 2];
        lam2[0] = 0.0;
        lam2[N - 1] = 0.0;
        for (int64_t i = 1; i < N - 1; ++i)
            lam2[i] = eq3(lam[i + 1], lam[i], lam[i - 1], r, w);
        double *t = lam; lam = lam2; lam2 = t;
    }
    memcpy(grad_u0, lam, (size_t)N * sizeof(double));
    *grad_r = gr;
    if (grad_c1) *grad_c1 = gc1;
    if (grad_cN) *grad_cN = gcN;
    free(traj);
    free(seg);
    free(lam);
    free(lam2);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */
/* Discrete adjoint of the emulated asynchronous iteration (Eq.4 with its      */
/* seeded delay schedule, Dirichlet ends), derived from Eq.4.                   */
/*                                                                              */
/* For a fixed schedule the step is u_i(k+1) = (1-2r) u_i(k)                    */
/*   + r u_{i-1}(sL(i,k)) + r u_{i+1}(sR(i,k)), i = 1..N-2, where sL, sR are k    */
/* for reads inside a subdomain and max(0, k - delta) across a subdomain edge;  */
/* u_0(k) = c1 and u_{N-1}(k) = cN for every k.  Reverse mode, step by step from */
/* k = K-1 down to 0, each term sending r or (1-2r) times lambda_i(k+1) back to  */
/* the state it read (the delay schedule reversed):                              */
/*   lambda_i(k)            += (1-2r) lambda_i(k+1)                              */
/*   lambda_{i-1}(sL(i,k))  += r lambda_i(k+1)   (to dL/dc1 when i-1 = 0)         */
/*   lambda_{i+1}(sR(i,k))  += r lambda_i(k+1)   (to dL/dcN when i+1 = N-1)       */
/*   dL/dr += lambda_i(k+1) (u_{i-1}(sL) + u_{i+1}(sR) - 2 u_i(k))                */
/* starting from lambda(K) = gK with its end entries moved to dL/dc1, dL/dcN.    */
/* dL/du0 = lambda(0) with ends 0.  The whole forward trajectory and all        */
/* lambda(k) are kept (small rods only).  If scales != NULL it receives the     */
/* magnitudes that bound the rounding of the three scalar sums:                  */
/*   scales[0] = sum_k sum_i |lambda_i(k+1)| (|u_{i-1}(sL)| + |u_{i+1}(sR)|       */
/*               + 2 |u_i(k)|),                                                   */
/*   scales[1] = scales[2] = r sum_{k=1..K} max_i |lambda_i(k)|.                  */
/* ------------------------------------------------------------------------- */
/* The same with the delay schedule `kind` of oracle_sched_delay. */
int oracle_async_adjoint_kind(int64_t N, int64_t P, const double *u_in, const double *gK,
                              double r, double c1, double cN, int64_t K, int d, uint64_t seed,
                              int kind, double *grad_u0, double *grad_r, double *grad_c1,
                              double *grad_cN, double *scales)
{
    if (N < 3 || K < 0 || !r_is_valid(r) || d < 0 || P < 1 || P > N || kind < 0 || kind > 2)
        return ORACLE_EINVAL;
    double *u = (double *)malloc((size_t)((K + 1) * N) * sizeof(double));
    double *lam = (double *)calloc((size_t)((K + 1) * N), sizeof(double));
    int64_t *sub = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    if (!u || !lam || !sub) { free(u); free(lam); free(sub); return ORACLE_ENOMEM; }
    for (int64_t i = 0, p = 0; i < N; ++i) {
        while (p + 1 < P && sub_lo(p + 1, N, P) <= i) ++p;
        sub[i] = p;
    }
    /* the step each interior point reads its left / right neighbour at */
#define DELAY(k, p, side) oracle_sched_delay(kind, seed, k, p, side, P, d)
#define READ_L(i, k) ((sub[i] > 0 && (i) == sub_lo(sub[i], N, P)) \
                      ? ((k) - DELAY(k, sub[i], 0) < 0 ? 0 : (k) - DELAY(k, sub[i], 0)) \
                      : (k))
#define READ_R(i, k) ((sub[i] < P - 1 && (i) == sub_lo(sub[i] + 1, N, P) - 1) \
                      ? ((k) - DELAY(k, sub[i], 1) < 0 ? 0 : (k) - DELAY(k, sub[i], 1)) \
                      : (k))
    const double w = 1.0 - 2.0 * r;
    /* forward, keeping every state */
    memcpy(u, u_in, (size_t)N * sizeof(double));
    u[0] = c1;
    u[N - 1] = cN;
    for (int64_t k = 0; k < K; ++k) {
        double *nxt = u + (k + 1) * N;
        nxt[0] = c1;
        nxt[N - 1] = cN;
        for (int64_t i = 1; i < N - 1; ++i) {
            const double left = u[READ_L(i, k) * N + i - 1];
            const double right = u[READ_R(i, k) * N + i + 1];
            nxt[i] = eq3(right, u[k * N + i], left, r, w);
        }
    }
    /* backward */
    double gc1 = gK[0], gcN = gK[N - 1], gr = 0.0, sr = 0.0, sl = 0.0;
    for (int64_t i = 1; i < N - 1; ++i) lam[K * N + i] = gK[i];
    for (int64_t k = K - 1; k >= 0; --k) {
        double lmax = 0.0;
        for (int64_t i = 1; i < N - 1; ++i) {
            const double l = lam[(k + 1) * N + i];
            const int64_t rl = READ_L(i, k), rr = READ_R(i, k);
            const double left = u[rl * N + i - 1], right = u[rr * N + i + 1];
            gr += l * (left + right - 2.0 * u[k * N + i]);
            sr += fabs(l) * (fabs(left) + fabs(right) + 2.0 * fabs(u[k * N + i]));
            if (fabs(l) > lmax) lmax = fabs(l);
            lam[k * N + i] += w * l;
            if (i - 1 == 0) gc1 += r * l;
            else lam[rl * N + i - 1] += r * l;
            if (i + 1 == N - 1) gcN += r * l;
            else lam[rr * N + i + 1] += r * l;
        }
        sl += r * lmax;
    }
#undef READ_L
#undef READ_R
#undef DELAY
    for (int64_t i = 0; i < N; ++i) grad_u0[i] = (i == 0 || i == N - 1) ? 0.0 : lam[i];
    *grad_r = gr;
    *grad_c1 = gc1;
    *grad_cN = gcN;
    if (scales) {
        scales[0] = sr;
        scales[1] = sl;
        scales[2] = sl;
    }
    free(u);
    free(lam);
    free(sub);
    return ORACLE_OK;
}

int oracle_async_adjoint(int64_t N, int64_t P, const double *u_in, const double *gK, double r,
                         double c1, double cN, int64_t K, int d, uint64_t seed, double *grad_u0,
                         double *grad_r, double *grad_c1, double *grad_cN, double *scales)
{
    return oracle_async_adjoint_kind(N, P, u_in, gK, r, c1, cN, K, d, seed, 0, grad_u0, grad_r,
                                     grad_c1, grad_cN, scales);
}

/*
 * The same adjoint on the periodic ring of Section 5.3 (reading of the ends as
 * in async_run_periodic): every point is updated, its neighbours wrap around,
 * and with P > 1 every subdomain edge reads across with a delay.  No end
 * values, so only dL/du0 (every point) and dL/dr; scales[0] as above.
 */
int oracle_async_adjoint_periodic(int64_t N, int64_t P, const double *u_in, const double *gK,
                                  double r, int64_t K, int d, uint64_t seed, double *grad_u0,
                                  double *grad_r, double *scales)
{
    if (N < 3 || K < 0 || !r_is_valid(r) || d < 0 || P < 1 || P > N) return ORACLE_EINVAL;
    double *u = (double *)malloc((size_t)((K + 1) * N) * sizeof(double));
    double *lam = (double *)calloc((size_t)((K + 1) * N), sizeof(double));
    int64_t *sub = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    if (!u || !lam || !sub) { free(u); free(lam); free(sub); return ORACLE_ENOMEM; }
    for (int64_t i = 0, p = 0; i < N; ++i) {
        while (p + 1 < P && sub_lo(p + 1, N, P) <= i) ++p;
        sub[i] = p;
    }
    const double w = 1.0 - 2.0 * r;
    /* the steps point i reads its left and right neighbours at, during step k */
    int64_t *rl = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    int64_t *rr = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    if (!rl || !rr) { free(u); free(lam); free(sub); free(rl); free(rr); return ORACLE_ENOMEM; }
    memcpy(u, u_in, (size_t)N * sizeof(double));
    /* forward, keeping every state and nothing else: the read steps are
     * recomputed in the backward sweep from the same schedule */
    for (int64_t k = 0; k < K; ++k) {
        const double *cur = u + k * N;
        double *nxt = u + (k + 1) * N;
        for (int64_t i = 0; i < N; ++i) {
            const int64_t il = (i == 0) ? N - 1 : i - 1, ir = (i == N - 1) ? 0 : i + 1;
            int64_t sl = k, sr = k;
            if (P > 1 && i == sub_lo(sub[i], N, P)) {
                sl = k - oracle_delay(seed, k, sub[i], 0, P, d);
                if (sl < 0) sl = 0;
            }
            if (P > 1 && i == sub_lo(sub[i] + 1, N, P) - 1) {
                sr = k - oracle_delay(seed, k, sub[i], 1, P, d);
                if (sr < 0) sr = 0;
            }
            nxt[i] = eq3(u[sr * N + ir], cur[i], u[sl * N + il], r, w);
        }
    }
    double gr = 0.0, sc = 0.0;
    for (int64_t i = 0; i < N; ++i) lam[K * N + i] = gK[i];
    for (int64_t k = K - 1; k >= 0; --k) {
        for (int64_t i = 0; i < N; ++i) {
            rl[i] = k;
            rr[i] = k;
            if (P > 1 && i == sub_lo(sub[i], N, P)) {
                rl[i] = k - oracle_delay(seed, k, sub[i], 0, P, d);
                if (rl[i] < 0) rl[i] = 0;
            }
            if (P > 1 && i == sub_lo(sub[i] + 1, N, P) - 1) {
                rr[i] = k - oracle_delay(seed, k, sub[i], 1, P, d);
                if (rr[i] < 0) rr[i] = 0;
            }
        }
        for (int64_t i = 0; i < N; ++i) {
            const int64_t il = (i == 0) ? N - 1 : i - 1, ir = (i == N - 1) ? 0 : i + 1;
            const double l = lam[(k + 1) * N + i];
            const double left = u[rl[i] * N + il], right = u[rr[i] * N + ir];
            gr += l * (left + right - 2.0 * u[k * N + i]);
            sc += fabs(l) * (fabs(left) + fabs(right) + 2.0 * fabs(u[k * N + i]));
            lam[k * N + i] += w * l;
            lam[rl[i] * N + il] += r * l;
            lam[rr[i] * N + ir] += r * l;
        }
    }
    memcpy(grad_u0, lam, (size_t)N * sizeof(double));
    *grad_r = gr;
    if (scales) scales[0] = sc;
    free(u);
    free(lam);
    free(sub);
    free(rl);
    free(rr);
    return ORACLE_OK;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
