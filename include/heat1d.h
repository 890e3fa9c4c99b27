/*
 * heat1d.h -- C ABI of libheat1d.so, the gfx950 (MI355X) implementation of the
 * explicit heat-equation update of Lee and Bhattacharya, "Asynchronous Parallel
 * Computing Algorithm implemented in 1D Heat Equation with CUDA"
 * (arXiv:1510.08982).
 *
 * The method (Section 2, Eq.3): on N grid points with Dirichlet ends
 *     u_0(k) = c1,  u_{N-1}(k) = cN   for every k,
 * every interior point advances by
 *     u_i(k+1) = r u_{i+1}(k) + (1-2r) u_i(k) + r u_{i-1}(k),   0 < r <= 1/2.
 * The asynchronous form (Section 3, Eq.4) splits the rod into subdomains
 * (processing elements); the two points of a subdomain that border another
 * subdomain read that neighbour's value from one of the last q steps instead of
 * step k.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Indexing is 0-based: the paper's point i is point i-1 here, so the ends are
 *    points 0 and N-1.  Whatever u0 holds at the ends is ignored and replaced by
 *    c1 / cN (Section 2: the ends hold "for all k", including k = 0).
 *  - Precision: HEAT1D_F32 arrays hold float, HEAT1D_F64 arrays hold double.
 *    The scalar arguments r, c1, cN are passed as double and rounded to the
 *    array precision once.  Every kernel evaluates one step as
 *    c + r*((a + b) - 2c) with fused multiply-adds (algebraically Eq.3), so all
 *    kernels of one precision produce bitwise-identical results.
 *  - Memory: every array argument is a DEVICE pointer owned by the caller,
 *    except where a parameter name ends in _host.  Arrays are dense and
 *    contiguous.  The library never allocates device memory; scratch space is
 *    the caller's `workspace`, whose size the matching *_workspace_bytes call
 *    returns (256-byte alignment required), except for
 *    heat1d_run_async_noalloc, whose scratch is a fixed array the library
 *    holds on each device.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = default
 *    stream).  All work is enqueued on it; no call synchronises the host except
 *    the autotuners, heat1d_async_status, heat1d_batched_prepare and
 *    heat1d_last_kernel_ms.
 *  - Errors: argument errors are detected before anything is enqueued and are
 *    returned as a status code; nothing is written in that case.  Device-side
 *    errors (watchdog time-out of the asynchronous kernel) are recorded in the
 *    workspace and reported by heat1d_async_status after the stream has
 *    finished.
 *  - Thread safety: a plan may be used from one host thread at a time.  Two
 *    concurrent calls must not share a workspace.
 */
#ifndef HEAT1D_H
#define HEAT1D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
enum heat1d_status {
    HEAT1D_OK = 0,
    HEAT1D_EINVAL = 1,       /* an argument is out of range or a pointer is NULL */
    HEAT1D_EUNSUPPORTED = 2, /* valid request the library does not implement    */
    HEAT1D_EOCCUPANCY = 3,   /* persistent kernel cannot keep all workgroups resident */
    HEAT1D_ETIMEOUT = 4,     /* asynchronous kernel watchdog expired              */
    HEAT1D_EHIP = 5,         /* a HIP runtime call failed                         */
    HEAT1D_ESCRATCH = 6      /* heat1d_run_async_noalloc: the run needs more scratch
                                than the library's fixed array holds              */
};

enum heat1d_dtype { HEAT1D_F32 = 0, HEAT1D_F64 = 1 };

/* Synchronous kernel choice (heat1d_opts.sync_kernel). */
enum heat1d_sync_kernel {
    HEAT1D_SYNC_AUTO = 0,     /* plan's default, or the autotuner's choice        */
    HEAT1D_SYNC_STEP = 1,     /* one launch per step, two global buffers          */
    HEAT1D_SYNC_TILED = 2,    /* depth-T temporal blocking, T steps per launch    */
    HEAT1D_SYNC_RESIDENT = 3, /* whole rod in one workgroup's registers, K steps  */
    HEAT1D_SYNC_PIPELINED = 4  /* TILED with persistent wavefronts that load the
                                 next tile while computing the current one; same
                                 results bit for bit.  A pass whose buffers are
                                 not 16-byte aligned, whose N is not a multiple
                                 of 4 (FP32) / 2 (FP64), or whose rod fits one
                                 tile runs the TILED kernel instead            */
};

/* Asynchronous read policy (heat1d_run_async `mode`). */
enum heat1d_async_mode {
    HEAT1D_ASYNC_EMULATED = 0, /* replay the seeded delay schedule exactly        */
    HEAT1D_ASYNC_HARDWARE = 1  /* read the newest published value, at most d old  */
};

/* Boundary of the rod (heat1d_opts `boundary`). */
enum heat1d_boundary {
    HEAT1D_BC_DIRICHLET = 0, /* u_0 = c1, u_{N-1} = cN at every step (Section 2)      */
    HEAT1D_BC_PERIODIC = 1   /* the two ends are neighbours: a ring of N points
                                (Section 5.3); run by heat1d_run_sync and
                                heat1d_autotune_sync (one launch per step, or
                                ring tiles: sync_kernel TILED with depth_t,
                                pts_per_lane, fuse_steps and waves wavefronts
                                per tile, the same tile shapes as the Dirichlet
                                rod's; RESIDENT and PIPELINED give
                                HEAT1D_EUNSUPPORTED at plan creation), by
                                heat1d_run_sync_observed (norms of the whole
                                ring), by heat1d_run_async(_noalloc) with nsub >= 2
                                (subdomains 0 and P-1 are neighbours), by
                                heat1d_run_async_ensemble(_snapshots), by
                                heat1d_run_async_ensemble_adjoint and by
                                heat1d_run_async_adjoint (nsub >= 2); every other
                                entry point returns HEAT1D_EUNSUPPORTED          */
};

/* Plan options.  Zero in any field means "default / let the plan decide". */
typedef struct heat1d_opts {
    int32_t sync_kernel;      /* enum heat1d_sync_kernel                            */
    int32_t depth_t;          /* tiled kernel: steps per pass T (1..256)             */
    int32_t pts_per_lane;     /* points held per lane (tiled / resident / async).  On a
                                 plan with nsub > 0 and sync_kernel AUTO, waves and
                                 pts_per_lane shape the asynchronous kernel only and
                                 the synchronous kernel keeps its defaults           */
    int32_t waves;            /* resident / async: wavefronts per workgroup (1..16);
                                 TILED: wavefronts per tile (1, or 4 or 8: one tile
                                 per workgroup, wavefront boundaries traded through
                                 LDS once per sweep, 1/4 or 1/8 of the halo work;
                                 bit for bit TILED's results when fuse_steps = 1) */
    int32_t nsub;             /* async: number of subdomains P                       */
    int32_t max_delay;        /* async: largest d a run may use (sizes the halo ring; default 16) */
    int64_t watchdog_polls;   /* async: polls of a neighbour flag before giving up (default 2^22) */
    int32_t ckpt_stride;      /* adjoint: steps between checkpoints (default ceil(sqrt K) rounded
                                 up to a multiple of the sub-stretch, 24 steps FP32, 16 FP64) */
    int32_t nrods;            /* sync / adjoint: equal rods stacked back to back (default 1) */
    int32_t fuse_steps;       /* TILED / PIPELINED: steps S per register sweep on tiles that
                                 hold no rod end (1, 2 or 4, and 8 on FP32 wide tiles of
                                 16 or 32 points per lane; 0 = 1, and lets the autotuner
                                 try the others).  S > 1 applies the S-step stencil, the S-th
                                 power of Eq.3's three-point stencil: the same iteration
                                 with fewer roundings, so results differ from S = 1 in the
                                 last bits (within the stated tolerances), while tiles
                                 holding a rod end still take single steps            */
    int32_t jitter;           /* async: each workgroup pauses a seeded 0..jitter short sleeps
                                 (about 64 clocks each) per step, drawn from the run's
                                 seed, to perturb the timing: it provokes staleness in
                                 hardware mode and must not change an emulated run's
                                 result (0 = none; at most 65536)                      */
    int32_t boundary;         /* enum heat1d_boundary; default: Dirichlet ends          */
    int32_t grad_sum;         /* adjoint: 0 = grad_r (heat1d_backward_checkpointed,
                                 heat1d_adjoint) and grad_c1, grad_cN (heat1d_adjoint_ends)
                                 hold one double per rod; 1 = the rods share the plan's
                                 single r, c1 and cN, and each of those outputs is ONE
                                 double, the derivative with respect to that shared
                                 value: the per-rod sensitivities summed in double in
                                 a fixed order (the same bits on every run)          */
    int32_t delay_schedule;   /* emulated asynchronous runs (heat1d_run_async(_noalloc),
                                 heat1d_run_async_adjoint): which of the d+1 allowed
                                 values each subdomain-edge read takes (Eq.4): 0 = the
                                 seeded draw (default), 1 = always the oldest (delay d),
                                 2 = delay d on odd steps and 0 on even ones; the
                                 ensemble entry points and periodic plans take 0
                                 only (else HEAT1D_EUNSUPPORTED)                     */
} heat1d_opts;

typedef struct heat1d_plan_s *heat1d_plan_t;

/* ---- plans ---------------------------------------------------------------- */

/* Create a plan for rods of N points (N >= 3) in precision `dtype`.  `opts`
 * may be NULL.  With opts->nrods = B > 1 the arrays hold B rods of N points
 * each, back to back, all advanced with the same r, c1, cN and K.
 * Returns HEAT1D_EINVAL for N < 3, a bad dtype, B < 1 or options out of range. */
int heat1d_plan_create(heat1d_plan_t *out, int64_t N, int32_t dtype, const heat1d_opts *opts);

/* Create a plan for a batch of `nrods` independent rods of uneven length.
 * N_host[b] >= 3 is the length of rod b and K_host[b] >= 0 its step count (both
 * host arrays, read during the call only; K_host is used to order the work,
 * longest first).  Every rod must fit one workgroup: N <= 65536 (F32) or
 * N <= 32768 (F64), else HEAT1D_EUNSUPPORTED. */
int heat1d_plan_batched(heat1d_plan_t *out, int32_t nrods, const int64_t *N_host,
                        const int32_t *K_host, int32_t dtype, const heat1d_opts *opts);

void heat1d_plan_destroy(heat1d_plan_t plan);

/* Bytes of workspace each call needs.  For the sync path this is one state
 * (N*B elements); the async path adds its halo ring and flags; the adjoint adds
 * its checkpoints for K steps; the batched path holds its work queues. */
size_t heat1d_sync_workspace_bytes(heat1d_plan_t plan);  /* any sync kernel */
size_t heat1d_async_workspace_bytes(heat1d_plan_t plan);
size_t heat1d_adjoint_workspace_bytes(heat1d_plan_t plan, int64_t K);
size_t heat1d_batched_workspace_bytes(heat1d_plan_t plan);

const char *heat1d_strerror(int status);

/* Human-readable description of the plan's current kernel choice (static
 * storage inside the plan; valid until the plan changes or is destroyed). */
const char *heat1d_plan_describe(heat1d_plan_t plan);

/* ---- synchronous iteration (Section 2, Eq.3) ------------------------------ */

/* u(K) from u0 by K steps of Eq.3 with Dirichlet ends c1 (point 0) and cN
 * (point N-1).  u0 and uK hold N*B elements and must not overlap; u0 is not
 * modified.  K = 0 copies u0 with its ends replaced.  r must lie in (0, 0.5]
 * (Section 2 stability range); K >= 0.  On a periodic plan every point is
 * updated, point 0 and point N-1 being neighbours (Section 5.3); c1 and cN are
 * not used and K = 0 copies u0. */
int heat1d_run_sync(heat1d_plan_t plan, const void *u0, void *uK, double r, double c1,
                    double cN, int64_t K, void *workspace, void *stream);

/* Time every candidate synchronous kernel configuration on the caller's
 * buffers for `K_probe` steps, keep the fastest in the plan and return its
 * time in *best_ms (may be NULL).  Synchronises `stream`.  uK is overwritten. */
int heat1d_autotune_sync(heat1d_plan_t plan, const void *u0, void *uK, double r, int64_t K_probe,
                         void *workspace, void *stream, double *best_ms);

/* Observable of the run (the history of states the asynchronous code of
 * Section 4 keeps, and Section 5.1 plots, reduced to one number per state):
 * heat1d_run_sync, and in addition norms[b*(K/every + 1) + j] = ||u_b(j*every)||_2
 * for j = 0 .. K/every and each rod b (the 2-norm over all N points, ends
 * included; u(0) with its ends replaced; on a periodic plan every point as
 * the ring holds it, c1 and cN unused).  norms: B*(K/every + 1) doubles in
 * device memory, written in a fixed summation order (the same bits on every
 * run); it must not overlap the other buffers.  every >= 1.  The state after
 * each multiple of `every` steps is the plan's own kernel's, so uK equals
 * heat1d_run_sync's for the same plan when `every` is a multiple of the
 * plan's pass depth (else the passes are cut at the multiples of `every`).
 * workspace: heat1d_observed_workspace_bytes(plan) bytes. */
size_t heat1d_observed_workspace_bytes(heat1d_plan_t plan);
int heat1d_run_sync_observed(heat1d_plan_t plan, const void *u0, void *uK, double r, double c1,
                             double cN, int64_t K, int64_t every, double *norms, void *workspace,
                             void *stream);

/* ---- asynchronous iteration (Section 3, Eq.4) ----------------------------- */

/* u(K) by Eq.4 with P = opts.nsub subdomains, subdomain p owning points
 * [floor(pN/P), floor((p+1)N/P)).  Inside a subdomain every read is current;
 * the first (last) point of a subdomain reads its left (right) neighbour
 * subdomain's edge value from step k - delta with 0 <= delta <= d (q = d+1 in
 * the paper's notation).  Each subdomain is owned by one workgroup of a
 * persistent kernel; there is no grid-wide barrier.
 *   mode HEAT1D_ASYNC_EMULATED: delta = the seeded schedule
 *     delta(k,p,side) = ((x >> 32) * (d+1)) >> 32,
 *     x = sm64(seed ^ sm64(((k*P + p) << 1) | side)), sm64 = SplitMix64 output
 *     function; reads before step 0 read step 0.  Deterministic.
 *   mode HEAT1D_ASYNC_HARDWARE: the workgroup uses the newest value its
 *     neighbour has published (never newer than step k) and waits only while
 *     that value would be older than k - d.  Not reproducible run to run.
 * `stats` (may be NULL): int64 device array of d+3 entries, incremented by the
 * run: [0..d] = histogram of the delays actually used, [d+1] = total polls of
 * neighbour flags, [d+2] = number of edge reads.
 * Requires 1 <= P <= N/2, 0 <= d <= opts.max_delay, and that all P workgroups
 * fit on the device at once (else HEAT1D_EOCCUPANCY).
 * On a periodic plan (HEAT1D_BC_PERIODIC, Section 5.3) the rod is a ring: c1
 * and cN are unused, every point is updated, the first point of subdomain 0
 * reads the last point of subdomain P-1 with the delay of (k, 0, left) and the
 * last point of P-1 reads point 0 with the delay of (k, P-1, right); P >= 2
 * (P = 1 gives HEAT1D_EUNSUPPORTED: nothing would be delayed, which is
 * heat1d_run_sync's ring). */
int heat1d_run_async(heat1d_plan_t plan, const void *u0, void *uK, double r, double c1,
                     double cN, int64_t K, int32_t d, uint64_t seed, int32_t mode,
                     void *workspace, int64_t *stats, void *stream);

/* Allocation-free variant of heat1d_run_async, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same run, same kernels and same
 * results bit for bit, with the halo ring, progress hints and status words in
 * a fixed array the library owns (HEAT1D_NOALLOC_SCRATCH_BYTES = 4 MiB per
 * device, held until the process ends) instead of a workspace.  The call
 * allocates nothing: no hipMalloc, hipFree or allocating library routine.
 * Arguments and checks as heat1d_run_async, without `workspace`, plus
 * `status`: NULL or a caller-owned device int32 that receives the run's
 * watchdog status (HEAT1D_OK or HEAT1D_ETIMEOUT) when the stream reaches the
 * end of the run.  A plan whose heat1d_async_workspace_bytes exceeds
 * HEAT1D_NOALLOC_SCRATCH_BYTES is refused with HEAT1D_ESCRATCH before anything
 * is enqueued (FP32: P subdomains x (2 max_delay + 2) x 16 bytes + P x 8 bytes
 * + 512 bytes, rounded up to 256 bytes; P = 1024 at max_delay = 16 uses 0.55
 * MiB).  Every call on one device shares that device's array and leaves the
 * last run's contents in it; the run re-initialises what must start fresh.
 * Two calls whose runs overlap in time on one device (two streams, two host
 * threads) race on the array and give undefined results: serialise them. */
#define HEAT1D_NOALLOC_SCRATCH_BYTES ((size_t)4 << 20)
int heat1d_run_async_noalloc(heat1d_plan_t plan, const void *u0, void *uK, double r, double c1,
                             double cN, int64_t K, int32_t d, uint64_t seed, int32_t mode,
                             int64_t *stats, int32_t *status, void *stream);

/* Status of the last asynchronous run on `workspace` (synchronises `stream`):
 * HEAT1D_OK or HEAT1D_ETIMEOUT. */
int heat1d_async_status(heat1d_plan_t plan, void *workspace, void *stream);

/* The emulated schedule itself: out[(k*P + p)*2 + side] = delta(k, p, side)
 * for k < K, p < P, side 0 (left edge) / 1 (right edge); uint8 device array. */
int heat1d_delay_schedule(int32_t P, int64_t K, int32_t d, uint64_t seed, uint8_t *out,
                          void *stream);

/* ---- ensemble of emulated asynchronous runs ------------------------------- */

/* Section 5, Fig. 3: many runs of the same rod whose trajectories differ only
 * through their random delays, each with the 2-norm of its state over time.
 * One launch runs the E = opts.nrods members of a plan for rods of N points,
 * cut into P = opts.nsub subdomains (0 means P = N: one grid point per
 * subdomain, the set-up of the paper's experiment; 1 <= P <= N).  Member e
 * iterates Eq.4 in the emulated mode of heat1d_run_async -- delays drawn from
 * the same seeded schedule, here with the seed seeds[e] -- from
 * u0[e*N .. e*N+N-1] (ends replaced by c1, cN) for K steps and leaves u(K) in
 * uK[e*N ..].  If `norms` is not NULL, norms[e*(K/every + 1) + j] receives the
 * 2-norm of the member's whole state (ends included) after j*every steps,
 * j = 0 .. K/every (squares summed in double precision, in a fixed order).
 * With opts.boundary = HEAT1D_BC_PERIODIC the rods are rings (Section 5.3,
 * Fig. 6): every point is updated, point 0 and point N-1 are neighbours, with
 * P > 1 every subdomain has two delayed edges, and c1, cN are not used.
 *
 * u0, uK: E*N elements (device); seeds: E uint64 values (device); norms: device
 * doubles or NULL.  No workspace: a member's last d+2 states and, for d > 0,
 * two rows of one delay byte per subdomain edge live in on-chip memory, so
 * (d+2)*N*elem + (d > 0 ? 4*P : 0) + 128 bytes (each term rounded up to a
 * multiple of 8) must not exceed 65536, else HEAT1D_EUNSUPPORTED; at d = 3
 * that is N <= 1633 FP64 / 3267 FP32 with P = 16, N <= 1486 / 2725 with P = N.
 * HEAT1D_EINVAL: NULL u0/uK/seeds, r outside (0, 0.5], K < 0, d outside
 * 0..255, every < 1, P > N, a batched plan, or overlapping buffers. */
int heat1d_run_async_ensemble(heat1d_plan_t plan, const void *u0, void *uK, double r,
                              double c1, double cN, int64_t K, int32_t d,
                              const uint64_t *seeds, int32_t every, double *norms,
                              void *stream);

/* heat1d_run_async_ensemble that also reports the members' states at chosen
 * steps (Section 5.1, Fig. 2: snapshots of the temperature profile as the
 * asynchronous iteration flattens it).  steps_host: nsnap host int64 values,
 * strictly increasing, each in [0, K] (read during the call only; 1 <= nsnap
 * <= 64).  snaps: E*nsnap*N elements (device); snaps[(e*nsnap + j)*N + i] =
 * u_i(steps_host[j]) of member e, the whole rod (ends included; step 0 is u0
 * with its ends replaced), the same values the run itself computes.
 * HEAT1D_EINVAL as heat1d_run_async_ensemble, and for a bad step list, a NULL
 * snaps or snaps overlapping another buffer. */
int heat1d_run_async_ensemble_snapshots(heat1d_plan_t plan, const void *u0, void *uK, double r,
                                        double c1, double cN, int64_t K, int32_t d,
                                        const uint64_t *seeds, int32_t every, double *norms,
                                        const int64_t *steps_host, int32_t nsnap, void *snaps,
                                        void *stream);

/* Gradients through the ensemble's emulated asynchronous runs (derived from
 * Eq.4 with the delay schedule fixed by each member's seed).  For member e
 * with dL/du(K) = gK[e*N ..], on a Dirichlet plan:
 *   lambda(K) = gK with both ends zeroed;
 *   lambda_j(k) = (1-2r) lambda_j(k+1) + r * (the lambda_{j+-1}(k'+1) of every
 *     step k' at which neighbour j+-1 read point j's value of step k: k' = k
 *     inside a subdomain, k' in k..k+d across a subdomain edge);
 *   dL/dr  = sum_k sum_j lambda_j(k+1) (u_{j-1}(sL) + u_{j+1}(sR) - 2 u_j(k)),
 *            sL, sR the steps the forward step read;
 *   dL/dc1 = gK[0]   + r sum_{k=1..K} lambda_1(k);
 *   dL/dcN = gK[N-1] + r sum_{k=1..K} lambda_{N-2}(k);
 *   dL/du0 = lambda(0) (ends 0).
 * On a periodic plan every point is updated and its neighbours wrap around:
 * lambda(K) = gK, the same recurrence over all N points, dL/du0 = lambda(0),
 * and grad_c1, grad_cN are written as 0 (the ring has no end values).
 * With d = 0 or P = 1 this is the adjoint of Eq.3.  One launch runs the
 * members forward (the same run as heat1d_run_async_ensemble, leaving every
 * state in `workspace` and u(K) in uK when uK is not NULL), a second one
 * reverses them.  grad_u0: E*N elements; grad_r, grad_c1, grad_cN: E doubles
 * each (device); the sums run in double, in a fixed order.  workspace:
 * heat1d_ensemble_adjoint_workspace_bytes(plan, K) bytes ((K+1)*N*E
 * elements).  On-chip limits as heat1d_run_async_ensemble, and also
 * (d+2)*N*elem + 2*N*elem + (d > 0 ? 2*(d+1)*N*elem + 2*(d+2)*P : 0) + 64
 * bytes (terms rounded up to a multiple of 8) <= 65536 (at d = 3, P = 16:
 * N <= 544 FP64 / 1088 FP32) and at most 4096 updated points, else
 * HEAT1D_EUNSUPPORTED.  HEAT1D_EINVAL as heat1d_run_async_ensemble, for NULL
 * gradients or workspace, and for any two of the buffers overlapping (u0 and
 * gK may). */
size_t heat1d_ensemble_adjoint_workspace_bytes(heat1d_plan_t plan, int64_t K);
int heat1d_run_async_ensemble_adjoint(heat1d_plan_t plan, const void *u0, const void *gK,
                                      double r, double c1, double cN, int64_t K, int32_t d,
                                      const uint64_t *seeds, void *uK, void *grad_u0,
                                      double *grad_r, double *grad_c1, double *grad_cN,
                                      void *workspace, void *stream);

/* Gradients through one emulated asynchronous run of a rod of any length
 * (derived from Eq.4 of Section 3, with the delay schedule of
 * heat1d_run_async's emulated mode fixed by `seed`): the run of
 * heat1d_run_async(plan, ..., mode = HEAT1D_ASYNC_EMULATED) on the plan's
 * nsub subdomains, then the recurrence stated for
 * heat1d_run_async_ensemble_adjoint (Dirichlet form) backwards from
 * lambda(K) = gK with its ends zeroed: dL/du0 = lambda(0) (ends 0), dL/dr,
 * dL/dc1 = gK[0] + r sum_k lambda_1(k), dL/dcN likewise.  On a periodic
 * plan (the ring of Section 5.3, nsub >= 2) the run is heat1d_run_async's
 * ring and the recurrence is the ring form stated for
 * heat1d_run_async_ensemble_adjoint: lambda(K) = gK, every point, neighbours
 * wrapping, grad_c1 = grad_cN = 0.  The forward pass
 * keeps u at every S-th step (S = opts.ckpt_stride, default ceil(sqrt(K)))
 * and, for the points next to the P-1 subdomain edges only, every step; the
 * backward pass replays each stretch of S steps from its checkpoint.  Both
 * run in lockstep, one launch per step: in the emulated mode the delays are a
 * fixed function of the seed, so the forward values equal those of
 * heat1d_run_async bit for bit.  u0, gK: N elements (device, read only; they
 * may alias); uK: NULL or N elements, receives u(K); grad_u0: N elements;
 * grad_r, grad_c1, grad_cN: one device double each, summed in double in a
 * fixed order.  workspace: heat1d_async_adjoint_workspace_bytes(plan, K)
 * bytes, about (K/S + S + 3) N elements plus 4 (K+1) P elements.
 * HEAT1D_EINVAL for NULL pointers, r outside (0, 1/2], K < 0, d outside
 * 0..255, non-finite ends, more subdomains than points or overlapping
 * buffers; HEAT1D_EUNSUPPORTED for a batched plan, nrods > 1, a periodic
 * plan with one subdomain, K >= 2^30 or N > 2^31 - 1. */
size_t heat1d_async_adjoint_workspace_bytes(heat1d_plan_t plan, int64_t K);
int heat1d_run_async_adjoint(heat1d_plan_t plan, const void *u0, const void *gK, double r,
                             double c1, double cN, int64_t K, int32_t d, uint64_t seed,
                             void *uK, void *grad_u0, double *grad_r, double *grad_c1,
                             double *grad_cN, void *workspace, void *stream);

/* ---- batched ragged rods -------------------------------------------------- */

/* Upload the plan's work order into `workspace`; needed once per workspace
 * before heat1d_run_batched (kept separate so that the run itself can be
 * captured in a HIP graph). */
int heat1d_batched_prepare(heat1d_plan_t plan, void *workspace, void *stream);

/* Advance every rod b of the batch by K[b] steps of Eq.3 in one persistent
 * launch.  Rod b occupies elements [offsets[b], offsets[b+1]) of u0 / uK
 * (offsets: int64 device array of nrods+1 entries, offsets[0] = 0, lengths
 * equal to the plan's N_host).  r, c1, cN: double device arrays (one per rod,
 * r in (0, 0.5]); K: int32 device array equal to the plan's K_host. */
int heat1d_run_batched(heat1d_plan_t plan, const void *u0, void *uK, const int64_t *offsets,
                       const double *r, const double *c1, const double *cN, const int32_t *K,
                       void *workspace, void *stream);

/* Choose the batched plan's work order by timing it on the caller's buffers:
 * the longest rod of the single-wavefront queue (0, 1/4, 1/2 or all of what
 * one wavefront holds) and of the 4-wavefront-group queue (none, 1/4, 1/2 or
 * all of what a group holds), then the number of workgroups that start with
 * those two queues (the plan's rule, 0, 1/8, 1/4, 1/2 or all of the grid).
 * Each candidate is timed as the better of two runs with HIP events; the
 * fastest is kept in the plan and uploaded into `workspace` (no further
 * heat1d_batched_prepare is needed for it; another workspace needs one).
 * Every candidate computes each rod with the same arithmetic, so results are
 * bit for bit those of the untuned plan.  A HIP graph captured before the
 * call holds the old queue lengths and must be captured again.  Arguments as
 * heat1d_run_batched;
 * uK is overwritten; synchronises `stream`; *best_ms (may be NULL) receives
 * the kept candidate's time. */
int heat1d_autotune_batched(heat1d_plan_t plan, const void *u0, void *uK, const int64_t *offsets,
                            const double *r, const double *c1, const double *cN,
                            const int32_t *K, void *workspace, void *stream, double *best_ms);

/* ---- discrete adjoint (derived from Eq.3) ---------------------------------- */

/* Forward K steps of Eq.3, also storing the states u(0), u(S), u(2S), ...
 * (S = checkpoint stride) in `workspace` for a later backward call.  The
 * passes use fused 4-step sweeps, so uK equals heat1d_run_sync's result to
 * within rounding (not bit for bit) and depends on S only through rounding.
 * uK may be NULL. */
int heat1d_forward_checkpointed(heat1d_plan_t plan, const void *u0, void *uK, double r,
                                double c1, double cN, int64_t K, void *workspace, void *stream);

/* Gradients of a loss L(u(K)) given gK = dL/du(K) (N*B elements), using the
 * checkpoints a preceding heat1d_forward_checkpointed call with the same
 * (r, c1, cN, K) left in `workspace`:
 *   lambda(K) = gK with both ends zeroed;
 *   lambda(k) = A^T lambda(k+1) (the same stencil with zero ends);
 *   dL/dr     = sum_k sum_i lambda_i(k+1) (u_{i+1}(k) - 2u_i(k) + u_{i-1}(k));
 *   dL/du0    = lambda(0) (ends 0).
 * The states inside each checkpoint stretch are recomputed.  grad_u0: N*B
 * elements (bit for bit independent of the checkpoint stride, given gK);
 * grad_r: B doubles (one per rod), or one double with opts.grad_sum = 1 (the
 * sum over rods, in a fixed order): per point the terms of one sub-stretch
 * (24 steps FP32, 16 FP64) are summed in the state precision, then per tile
 * and per rod in double precision, in a fixed order (deterministic: the same
 * bits on every run with the same plan). */
int heat1d_backward_checkpointed(heat1d_plan_t plan, const void *gK, double r, double c1,
                                 double cN, int64_t K, void *grad_u0, double *grad_r,
                                 void *workspace, void *stream);

/* dL/dc1 and dL/dcN for every rod b of the plan, given gK = dL/du(K):
 *   dL/dc1[b] = gK_b[0] + r sum_{k=1..K} lambda_{b,1}(k),
 *   dL/dcN[b] = gK_b[N-1] + r sum_{k=1..K} lambda_{b,N-2}(k)
 * (derived from Eq.3: the ends hold c1, cN at every step and only points 1 and
 * N-2 read them).  Computed without a backward sweep: u(K) is linear in
 * (u0, c1, cN), so dL/dc1[b] = <gK_b, w> with w = u(K) of one rod of the plan's
 * N and the given r from a zero interior with c1 = 1, cN = 0, and dL/dcN[b] =
 * <gK_b, w read back to front> (the mirror image of w is the response to cN);
 * one synchronous run of one rod serves every rod.  Sums in double, per
 * 8192-point chunk and per rod, in a fixed order.  grad_c1, grad_cN: nrods
 * doubles each (device), or one double each with opts.grad_sum = 1 (the sums
 * over rods, in a fixed order); workspace:
 * heat1d_adjoint_ends_workspace_bytes(plan).
 * HEAT1D_EINVAL for NULL pointers, r outside (0, 0.5], K < 0 or overlapping
 * buffers; HEAT1D_EUNSUPPORTED for a periodic plan or more than 65535 rods. */
size_t heat1d_adjoint_ends_workspace_bytes(heat1d_plan_t plan);
int heat1d_adjoint_ends(heat1d_plan_t plan, const void *gK, double r, int64_t K, double *grad_c1,
                        double *grad_cN, void *workspace, void *stream);

/* Both of the above: forward with checkpoints, then the backward sweep.
 * uK may be NULL. */
int heat1d_adjoint(heat1d_plan_t plan, const void *u0, const void *gK, double r, double c1,
                   double cN, int64_t K, void *grad_u0, double *grad_r, void *uK,
                   void *workspace, void *stream);

/* ---- introspection ---------------------------------------------------------- */

/* Average duration in milliseconds of the dominant kernel over the launches
 * enqueued by the most recent run call on this plan, measured with HIP events
 * on the launch stream when timing is enabled (heat1d_set_timing).  Returns a
 * negative value when nothing was timed.  Synchronises the last stream used. */
double heat1d_last_kernel_ms(heat1d_plan_t plan, int64_t *launches);

/* Enable (1) or disable (0) per-launch event timing of the dominant kernel. */
int heat1d_set_timing(heat1d_plan_t plan, int32_t enable);

/* The weights the fused S-step sweeps apply (heat1d_opts.fuse_steps = S in
 * {2, 4, 8}) for a step ratio r in (0, 0.5], as doubles w[0..S] (centre first):
 * u_i <- w[0] u_i + sum_{d=1..S} w[d] (u_{i-d} + u_{i+d}) stands for S steps
 * of Eq.3 (Section 2).  They are the coefficients of the S-th power of the
 * stencil (r', 1-2r', r') with r' = r rounded to the precision of `dtype`,
 * with the off-centre weights rounded to multiples of 2^-25 (FP32) / 2^-54
 * (FP64) and w[0] = 1 - 2 (w[1] + ... + w[S]), so that each is exact in that
 * precision and the row sum is exactly 1 (a constant state is a fixed point,
 * as for Eq.3 itself).  Host-only; no device is needed.  HEAT1D_EINVAL for a
 * bad dtype, r outside (0, 0.5], S not 2, 4 or 8, or w NULL. */
int heat1d_fused_weights(int32_t dtype, double r, int32_t S, double *w);

/* Library version string. */
const char *heat1d_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HEAT1D_H */
