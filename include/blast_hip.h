/*
 * blast_hip.h -- C ABI of the MI355X (gfx950) beyond-Limber C_ell library.
 *
 * The library evaluates, for every tomographic bin pair (i, j) and multipole l,
 *
 *   C^{AB}_ij(l) = N_AB(l) int dchi int_0^1 dR chi
 *                  [K_i^A(chi) K_j^B(R chi) + K_j^B(chi) K_i^A(R chi)] w^{AB}_l(chi, R chi)
 *
 * (Eq. final_cls of Chiarenza et al., arXiv:2410.03632, with the prefactors
 * N_gg = 2/pi, N_gs = (2/pi) sqrt((l+2)!/(l-2)!), N_ss = (2/pi) (l+2)!/(l-2)! of
 * Eqs. gg, gs, ss), where the projected matter density is the contraction
 *
 *   w^{AB}_l(chi1, chi2) = sum_n c_n(chi1, chi2) Ttilde^{AB}_{n;l}(chi1, chi2)      (Eq. pmd)
 *   Ttilde^{AB}_{n;l}    = int_{kmin}^{kmax} dk f^{AB}(k) T_n(x(k)) j_l(k chi1) j_l(k chi2)
 *                                                                                     (Eq. t_tilde)
 *
 * with f_gg = k^2, f_gs = 1, f_ss = 1/k^2, T_n the Chebyshev polynomials in
 * x(k) = 2 ln(k/kmin)/ln(kmax/kmin) - 1, and c_n the coefficients of the
 * polynomial that interpolates P at the first-kind Chebyshev points
 * (Eqs. chebpoints, a2, dft).  The outer integrals are quadrature sums over the
 * caller's chi nodes and R nodes (Sec. "The implementation").
 *
 * Conventions
 *  - Every entry point returns a blast_status and never throws or aborts.  On
 *    failure blast_last_error() returns a thread-local message.
 *  - "host" pointers are read during the call only.  "device" pointers are HIP
 *    device memory owned by the caller; the library never frees them.  Work is
 *    enqueued on the caller's stream (hipStream_t passed as void*, NULL = the
 *    null stream) and the call returns before it completes.
 *  - Multipoles are real values in [2, 4096] (blast_plan_desc.ell); they need
 *    not be integers.  Types: bit 1 = gg (clustering x clustering),
 *    bit 2 = gs (clustering x shear), bit 4 = ss (shear x shear).
 *  - Bins: n_g clustering bins first, then n_s shear bins.  Pair order of every
 *    output: gg (i <= j, row-major), then gs (i over clustering, j over shear),
 *    then ss (i <= j).
 *  - Kernels are the calligraphic K of Eq. final_cls: K = W for clustering and
 *    K = W / chi^2 for lensing.
 */
#ifndef BLAST_HIP_H
#define BLAST_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BLAST_OK = 0,
    BLAST_E_INVALID = 1,     /* bad argument, shape or grid                      */
    BLAST_E_OOM = 2,         /* device or host allocation failed / over budget   */
    BLAST_E_HIP = 3,         /* a HIP runtime call failed                        */
    BLAST_E_UNSUPPORTED = 4, /* valid request the library does not implement   */
    BLAST_E_BUSY = 5,        /* server queue full                                */
    BLAST_E_CANCELLED = 6    /* request cancelled                                */
} blast_status;

/* Arithmetic of the contraction (Eq. pmd).  FP64: FP64 basis, FP64 MFMA.
 * FP32: FP32 basis and coefficients, FP32 MFMA.  BF16: BF16 basis and
 * coefficients (per-row power-of-two scales), FP32 accumulate.  BF16X3: basis and
 * coefficients split into BF16 hi + lo parts, hi*hi + hi*lo + lo*hi, FP32
 * accumulate.  FP16X3: the same three products with FP16 hi + lo parts (about 22
 * significant bits per operand); every basis row and every row of the other operand
 * (one cosmology, one point) carries its own power-of-two scale that keeps its
 * magnitudes below 2^15, inside FP16's range (largest magnitude in [2^14, 2^15);
 * coefficients projected from nodal P: from the row's largest |P_j|, which bounds
 * |c_n| / 2, the projection running the same three products on P and the DCT matrix
 * split into FP16 hi + lo parts).  FP16X3 runs the fused contraction + R-quadrature
 * only: it needs nodal P with n_cheb % 4 == 0 in FP32 or n_cheb % 8 == 0 in FP64 (or P
 * given as coefficients), n_g + n_s <= 20 and no w_save, and is not available to the adjoint; other requests
 * are refused with BLAST_E_UNSUPPORTED.
 *
 * Nodal basis.  Since c = D P (Eq. dft, D the DCT-II matrix), the contraction
 * sum_n Ttilde_n c_n equals sum_j B_j P_j with B = Ttilde D; the plan keeps B next to
 * Ttilde and the forward contracts it with the nodal P values themselves, making and
 * storing no coefficients, when: FP16X3 on FP32 P with n_cheb % 4 == 0 and at most 16
 * bins (P rows split into FP16 hi + lo inside the contraction kernel; with 17-20 bins P is
 * split by the coefficient-input conversion instead of projected); FP32 on FP32 P with
 * n_cheb % 4 == 0 (P rows read in place of the padded coefficient rows); FP64 on FP64 P
 * with n_cheb a multiple of 32 (P rows are then laid out as the coefficient rows).  The backward on such calls computes dP = B^T dw likewise.  The
 * result is that of the projection route up to rounding; on the ridge R ~ 1 the terms
 * B_j P_j are quadrature weights of one sign, so the sum cancels far less than the
 * Chebyshev terms do and the error of the mixed paths drops on the named workloads
 * (figures below; on small grids with k up to 0.6/Mpc the two routes trade places, both
 * within 1e-4).  Other calls (FP64 P on FP32 or FP16X3, coefficient input, BF16 paths)
 * project per call.
 * The basis precompute is always FP64; the quadrature always accumulates in FP64.
 *
 * Accuracy.  The relative error of C against exact arithmetic on the same grids is about
 * u * kappa, where u is the relative error of one product of the contraction's operands and
 * kappa >= 1 is the cancellation of the problem: the ratio of the sum of the magnitudes of
 * the terms (Chebyshev or nodal terms of Eq. pmd, then the chi-R sum of Eq. final_cls) to
 * |C|.  kappa grows with the multipole and the Chebyshev order, and is largest for cross
 * spectra of well separated bins at high multipoles.  u is about 2^-52 (FP64), 2^-23 (FP32),
 * 2^-21 (FP16X3), 2^-15 (BF16X3: the hi*lo sum leaves 16 bits per operand) and 2^-7 (BF16: 8
 * bits per operand).  Measured against the FP64 oracle (element-wise, cross spectra floored at
 * 1e-3 of the geometric mean of the two auto spectra), nodal basis where it applies: at 20
 * multipoles on [2, 200] with 64 Chebyshev nodes FP64 8e-12, FP32 3.4e-6, FP16X3 1.5e-6,
 * BF16X3 9e-4, BF16 0.26; at 96 multipoles on [2, 1000] with 128 nodes FP64 4e-11, FP32
 * 4.4e-5, FP16X3 1.5e-5, BF16X3 9e-3, BF16 6.2 (through the per-call projection, on FP64 P:
 * FP32 3.1e-6 and 2.4e-4, FP16X3 1.4e-5 and 2.7e-4).  FP64 is the path for a 1e-6 bar and
 * FP16X3 or FP32 for 1e-3; BF16X3 meets 1e-3 only on grids like the first and stays within
 * 2e-2 on grids like the second; plain BF16 is not an accurate evaluation of C at either
 * (errors of order 1 at the second) and is kept to measure what the compensated split buys. */
typedef enum {
    BLAST_FP64 = 0,
    BLAST_FP32 = 1,
    BLAST_BF16 = 2,
    BLAST_BF16X3 = 3,
    BLAST_FP16X3 = 4
} blast_precision;

enum { BLAST_GG = 1, BLAST_GS = 2, BLAST_SS = 4 };

const char *blast_last_error(void);
const char *blast_version(void);

/* ------------------------------------------------------------------------- */
/* Grids (host only, no GPU).  Helpers that build the paper's default rules.  */
/* ------------------------------------------------------------------------- */

/* n evenly spaced chi nodes on [lo, hi] with composite Simpson weights
 * (Sec. "The implementation": Simpson rule on evenly spaced chi).  For an even n
 * the last three intervals use Simpson's 3/8 rule.  n >= 4.  Outputs: host [n]. */
blast_status blast_grid_chi_simpson(int32_t n, double lo, double hi, double *chi, double *w);

/* n first-kind Chebyshev points (Eq. chebpoints) mapped to [R_min, 1], ascending,
 * with Fejer's first-rule weights (the Clenshaw-Curtis-type rule for those
 * points; Sec. "The implementation").  0 <= R_min < 1.  Outputs: host [n]. */
blast_status blast_grid_R_fejer(int32_t n, double R_min, double *R, double *w);

/* The n first-kind Chebyshev points in ln k on [k_min, k_max] (Eqs. chebpoints,
 * cheb_pk), ascending in k: the k at which the caller samples P.  Output: host [n]. */
blast_status blast_grid_k_cheb(int32_t n, double k_min, double k_max, double *k);

/* ------------------------------------------------------------------------- */
/* Plan: grids + the resident, cosmology-independent basis (Eq. t_tilde)      */
/* ------------------------------------------------------------------------- */

typedef struct blast_plan blast_plan;

typedef struct {
    int32_t n_ell;
    const double *ell;    /* host [n_ell] multipoles, strictly increasing, in [2, 4096];
                             they need not be integers (the challenge's list is not):
                             an all-integer list takes one Bessel recurrence for all
                             orders, any other list one per distinct fractional part  */
    int32_t n_chi;
    const double *chi;    /* host [n_chi] chi nodes (> 0)                            */
    const double *w_chi;  /* host [n_chi] outer chi weights                          */
    int32_t n_R;
    const double *R;      /* host [n_R] R = chi2/chi1 nodes in (0, 1]                */
    const double *w_R;    /* host [n_R] R weights                                    */
    double k_min, k_max;  /* Chebyshev range, 0 < k_min < k_max                      */
    int32_t n_cheb;       /* Chebyshev nodes = coefficients, 2..128                  */
    uint32_t types;       /* subset of BLAST_GG | BLAST_GS | BLAST_SS                */
    uint32_t precisions;  /* bitmask of (1 << blast_precision) kept resident; FP64
                             is always built                                        */
    int32_t kq_panels;    /* k-quadrature: coarse panels uniform in arccos(x);
                             0 = n_cheb                                              */
    double kq_phase;      /* k-quadrature: max Bessel phase (chi1+chi2) dk per
                             16-point Gauss-Legendre sub-panel; 0 = 8                */
} blast_plan_desc;

/* Builds the grids and computes the basis on `device` in FP64 (synchronously),
 * then derives the other requested precisions.  The plan owns all of its device
 * memory.  Errors: INVALID (grids, ell list, sizes), OOM, HIP. */
blast_status blast_plan_create(const blast_plan_desc *desc, int32_t device, blast_plan **out);
blast_status blast_plan_destroy(blast_plan *plan);

/* Sizes: number of basis rows (types x ell), padded Chebyshev length, bytes of
 * resident basis per precision (host [5], indexed by blast_precision; FP64, FP32 and FP16X3
 * count their nodal basis too where the plan keeps one), k-quadrature node count, basis build
 * time in milliseconds.  Any output pointer may be NULL. */
blast_status blast_plan_info(const blast_plan *plan, int32_t *rows, int32_t *n_cheb_pad, size_t *basis_bytes,
                             int64_t *kq_nodes, double *build_ms);

/* Where to sample P: the k nodes (host [n_cheb], ascending). */
blast_status blast_plan_k_nodes(const blast_plan *plan, double *k);

/* The grids a plan was made with (useful after blast_plan_load).  Sizes and scalars are
 * written to the non-NULL pointers; the arrays (host, caller-owned, sized n_ell, n_chi,
 * n_chi, n_R, n_R) are filled when non-NULL. */
blast_status blast_plan_grids(const blast_plan *plan, int32_t *n_ell, int32_t *n_chi, int32_t *n_R,
                              int32_t *n_cheb, uint32_t *types, double *k_min, double *k_max, double *ell,
                              double *chi, double *w_chi, double *R, double *w_R);

/* Where to evaluate the kernels and P: chi_a (host [n_chi]) and R_b chi_a (host
 * [n_chi][n_R]).  Either pointer may be NULL. */
blast_status blast_plan_eval_points(const blast_plan *plan, double *chi, double *chi2);

/* Checkpoint of the cosmology-independent basis, which the method computes a single time
 * and reuses for every cosmology (Eq. t_tilde; Sec. "The implementation"): writes the grids and
 * the FP64 basis, followed by a 64-bit checksum of everything before it, to `path`.  The
 * file holds n_chi*n_R*rows_pad*n_cheb_pad doubles (several GB for a 256x96-point
 * 3x2pt grid).  Errors: INVALID (I/O), HIP. */
blast_status blast_plan_save(const blast_plan *plan, const char *path);

/* Rebuilds a plan from a file written by blast_plan_save on `device` without recomputing
 * the basis; `precisions` is a mask like the plan descriptor's, 0 meaning the saved set.
 * The reduced-precision copies are derived again on the device.  Errors: INVALID (not a
 * plan file, other version, truncated, checksum mismatch), OOM, HIP. */
blast_status blast_plan_load(const char *path, int32_t device, uint32_t precisions, blast_plan **out);

/* Copies the FP64 basis rows of one (chi_a, R_b) point to host:
 * out[t_slot * n_ell + l][n] for n < n_cheb (t_slot over the plan's types in the
 * order gg, gs, ss).  For tests and inspection. */
blast_status blast_plan_basis_point(const blast_plan *plan, int32_t a, int32_t b, double *out);

/* ------------------------------------------------------------------------- */
/* Forward: P grid + kernels -> C_ell for every bin pair                      */
/* ------------------------------------------------------------------------- */

typedef struct {
    int32_t batch;        /* number of independent cosmologies, >= 1              */
    int32_t precision;    /* blast_precision; must be resident in the plan        */
    int32_t p_dtype;      /* 0: P is FP64, 1: P is FP32                            */
    int32_t p_kind;       /* 0: P holds nodal values P(k_j, chi_a, R_b chi_a), k ascending
                             (blast_plan_k_nodes); 1: P holds the Chebyshev coefficients
                             c_n(chi_a, R_b chi_a) of Eq. cheb_pk (the projection is skipped) */
    const void *P;        /* device [batch][n_chi][n_R][n_cheb], 16-byte aligned (as
                             hipMalloc and torch allocations are; INVALID otherwise): read
                             in 16-byte pieces */
    int32_t n_g, n_s;     /* clustering / shear bins, n_g + n_s <= 32              */
    const double *K_chi;  /* device [batch][n_g+n_s][n_chi]: K at chi_a             */
    const double *K_chi2; /* device [batch][n_g+n_s][n_chi][n_R]: K at R_b chi_a    */
    uint32_t types;       /* subset of the plan's types                            */
    int32_t n_ell_out;    /* 0 = every plan multipole, else a subset:               */
    const int32_t *ell_idx; /* host [n_ell_out] increasing indices into the plan's ell */
    double *C;            /* device [batch][n_pairs][n_ell_out (or n_ell)]          */
    void *w_save;         /* device, nullable: [batch][n_chi*n_R][rows_pad] w of Eq. pmd
                             (FP64 for FP64, else FP32), rows as in blast_plan_basis_point */
    void *workspace;      /* device, nullable: caller scratch (blast_cl_workspace_bytes);
                             NULL = plan-owned scratch (then calls on one plan must not
                             overlap in time)                                        */
    size_t workspace_bytes;
    void *y_save;         /* device, nullable: [batch][rows_pad][n_chi][nbp] R-quadrature sums
                             Y[row][a][bin] = sum_b wR_b K_bin(R_b chi_a) w[a, b][row] (FP64 for
                             FP64, else FP32; nbp = 16 for at most 16 bins, else 32; bins past
                             n_g + n_s hold no values); a forward writes it, and a backward given
                             y_save of a forward with the same inputs reads it instead of summing
                             w again                                                        */
} blast_cl_args;

/* Device scratch for one forward or backward call with these sizes. */
blast_status blast_cl_workspace_bytes(const blast_plan *plan, int32_t batch, int32_t precision, int32_t n_bins,
                                      size_t *bytes);

/* Enqueues projection (Eq. dft) -> contraction (Eq. pmd) -> quadrature
 * (Eq. final_cls) on `stream`; calls that take the nodal basis (see the precisions
 * above) run no projection.  Errors: INVALID (shapes, types, precision not
 * resident), OOM (plan scratch), HIP. */
blast_status blast_cl_forward(blast_plan *plan, const blast_cl_args *args, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the computation of blast_cl_forward, with the call's
 * scratch in a fixed device array of 64 MiB that the library holds on every GPU it has made a
 * plan on, from then until the process ends, instead of plan-owned or caller memory.  The
 * caller passes inputs and outputs as for blast_cl_forward; args->workspace must be NULL.  The
 * call allocates nothing (no hipMalloc, no allocating library routine) and records no stage
 * timing.  A call whose scratch would exceed 64 MiB is refused with BLAST_E_UNSUPPORTED before
 * any work (the full 3x2pt grid with nodal P on 128 nodes fits one cosmology on every path).
 * All calls on one GPU share that GPU's array, which keeps the last call's contents: calls that
 * overlap in time on one GPU (other streams, other threads) race and must be serialised by the
 * caller.  Every byte of scratch a call reads it has written first, so nothing is cleared.
 * Errors: as blast_cl_forward; INVALID if args->workspace is set; HIP if the array's address on
 * this GPU could not be found when the plan was made. */
blast_status blast_cl_forward_noalloc(blast_plan *plan, const blast_cl_args *args, void *stream);

/* Adjoint of blast_cl_forward (reverse mode; not in the paper, whose conclusion lists
 * differentiability as future work).  With the same `args` (precision FP64 or FP32)
 * and dC = dL/dC (device, FP64, shaped like args->C) it enqueues on `stream`:
 *   dP      device, nullable, P's dtype and shape, 16-byte aligned: dL/dP (nodal values or
 *           coefficients per args->p_kind) -- the transposed contraction streams the basis again (on
 *           nodal P of the path's own type with n_cheb a multiple of 32 the nodal basis,
 *           whose product B^T dw is dP itself: FP64 reads the FP64 nodal basis, FP32 a
 *           transposed FP32 copy of it made at the first such call; otherwise Ttilde^T dw
 *           followed by the projection's adjoint);
 *   dK_chi  device, nullable, FP64 [batch][bins][n_chi]: dL/dK_chi;
 *   dK_chi2 device, nullable, FP64 [batch][bins][n_chi][n_R]: dL/dK_chi2.
 * args->C is not read.  args->w_save and args->y_save, if given, must hold w and Y of a
 * forward call with the same inputs.  w is read only for dK_chi2, and for dK_chi when
 * y_save is not given; without w_save a call that needs it recomputes w (projection and
 * contraction), and one that asks only for dP (or for dP and dK_chi with y_save) needs
 * neither.  Errors: INVALID, UNSUPPORTED (BF16 paths), OOM, HIP. */
blast_status blast_cl_backward(blast_plan *plan, const blast_cl_args *args, const double *dC, void *dP,
                               double *dK_chi, double *dK_chi2, void *stream);

/* ------------------------------------------------------------------------- */
/* Serving: continuous batching of single-cosmology requests                  */
/* ------------------------------------------------------------------------- */
/* The paper evaluates one data vector at a time and notes that running more
 * chains in parallel is the way to use a whole machine (Sec. "Discussion").  The
 * server turns independent requests (one cosmology each, with their own bins and
 * multipoles) into batched forward calls:
 *  - its device memory (hbm_budget) is split into `n_sets` slot-sets, each one arena with
 *    a stream of its own, so that a batch formed while others run overlaps with them;
 *  - a request's bins fall in a bucket: its clustering bins rounded up to a multiple of 4
 *    (at most max_g; 0 when it has none) and max_s shear bins.  A launch takes the bucket
 *    of its largest request; at creation a hipGraph is captured for every bucket and every
 *    batch size 1, 2, 4, ... up to `batch` whose inputs, outputs and forward scratch fit the
 *    arena (in the arena's layout for that shape), and a launch replays the smallest that
 *    holds its requests;
 *  - admission is by memory: a scheduler thread moves queued requests, in arrival order,
 *    into the forming set while the launch they would make still fits its arena, and
 *    launches the set when the next request does not fit, when its oldest request has
 *    waited max_wait_ms, or when no other set is running; requests complete as their set's
 *    event fires;
 *  - every launch computes all plan multipoles: the contraction streams basis rows in
 *    16-row tiles, and a request's multipoles are a subset spread over the plan's list, so
 *    it touches nearly every tile whatever its count; the requested ones are picked out;
 *  - each request's result depends only on its own inputs (per-cosmology arithmetic never
 *    mixes batch entries and a bucket only adds bins whose kernels are zero), so it is the
 *    same alone and in any mix.  The plan's memory (the basis) is fixed by its grids; the
 *    budget is the server's. */

typedef struct blast_server blast_server;

typedef struct {
    int32_t precision;    /* blast_precision resident in the plan                        */
    int32_t p_dtype;      /* dtype of request P: 0 FP64, 1 FP32                           */
    int32_t batch;        /* most requests per launch, >= 1                               */
    int32_t n_sets;       /* sets (concurrent batches), <= 4; 0 = as many as hbm_budget holds */
    int32_t max_g, max_s; /* largest clustering / shear bin counts a request may carry    */
    size_t hbm_budget;    /* device bytes the server may allocate; 0 = 8 GiB.  Each set gets
                             min(the bytes of `batch` requests of the largest bucket,
                             hbm_budget / n_sets)                                          */
    int32_t max_queue;    /* queued requests before submit returns BUSY; 0 = 4096         */
    double max_wait_ms;   /* launch a partly filled set after this wait                    */
    int32_t use_graphs;   /* 1: replay captured hipGraphs, 0: plain forward calls          */
} blast_server_desc;

typedef struct {
    const void *P;          /* host [n_chi][n_R][n_cheb] nodal P (p_dtype); read until completion */
    int32_t n_g, n_s;       /* bins of this request (<= max_g, max_s)                       */
    const double *K_chi;    /* host [n_g+n_s][n_chi]; read until completion                 */
    const double *K_chi2;   /* host [n_g+n_s][n_chi][n_R]; read until completion            */
    int32_t n_ell;          /* multipoles wanted (indices into the plan's ell, increasing)  */
    const int32_t *ell_idx; /* host [n_ell], copied at submit                               */
    double *C_out;          /* host [n_pairs(n_g, n_s)][n_ell]; written before completion   */
} blast_request;

typedef struct {
    int64_t submitted, completed, rejected, launches, queued, in_flight;
    double mean_fill;       /* mean requests per launch                                     */
    double p50_ms, p99_ms;  /* submit -> completion latency of completed requests           */
    double span_ms;         /* first submit -> last completion                              */
    int64_t cancelled;      /* requests cancelled before they ran                           */
    int64_t max_sets_in_flight; /* most sets running at once                                */
    int64_t n_sets;         /* sets created                                                 */
    int64_t set_bytes;      /* device bytes of one set's arena                              */
} blast_server_stats;

/* Errors: INVALID, OOM (the budget's share per set holds no request), UNSUPPORTED, HIP. */
blast_status blast_server_create(blast_plan *plan, const blast_server_desc *desc, blast_server **out);
/* Bytes of the arena a launch of `count` requests whose largest bins are (n_g, n_s) takes,
 * and (set_bytes, nullable) the bytes of one set's arena.  Errors: INVALID. */
blast_status blast_server_footprint(const blast_server *srv, int32_t n_g, int32_t n_s, int32_t count, size_t *bytes,
                                    size_t *set_bytes);
/* Queues a request.  BUSY when the queue is full, INVALID for a malformed request, OOM when a
 * launch of this request alone does not fit a set's arena. */
blast_status blast_server_submit(blast_server *srv, const blast_request *req, uint64_t *ticket);
/* Cancels a request that has not started: it completes at once with status BLAST_E_CANCELLED
 * (as wait or poll report).  BUSY if it is running (it will complete normally), INVALID if
 * the ticket is not pending. */
blast_status blast_server_cancel(blast_server *srv, uint64_t ticket);
/* Waits up to timeout_ms (< 0: forever) for a ticket.  Returns BUSY on timeout; on
 * completion writes the request's status and latency (either may be NULL) and forgets the
 * ticket. */
blast_status blast_server_wait(blast_server *srv, uint64_t ticket, int32_t timeout_ms, blast_status *req_status,
                               double *latency_ms);
/* Non-blocking wait: *done = 1 and the status and latency as wait writes them if the ticket
 * has completed (the ticket is then forgotten), else *done = 0. */
blast_status blast_server_poll(blast_server *srv, uint64_t ticket, int32_t *done, blast_status *req_status,
                               double *latency_ms);
blast_status blast_server_stats_get(blast_server *srv, blast_server_stats *stats);
/* Drains pending work, stops the scheduler and frees the server. */
blast_status blast_server_destroy(blast_server *srv);

/* ------------------------------------------------------------------------- */
/* Stage timing                                                               */
/* ------------------------------------------------------------------------- */

/* While enabled, blast_cl_forward records HIP events on the call's stream around
 * four intervals: 0 projection, 1 contraction, 2 R-quadrature, 3 chi-quadrature and
 * pair assembly.  On the mixed-precision paths without w_save, where the contraction
 * and the R-quadrature run fused, interval 1 holds the R-quadrature weight table and
 * interval 2 the fused kernel.  The events cost a few microseconds per call. */
blast_status blast_plan_profile(blast_plan *plan, int32_t enable);

/* ------------------------------------------------------------------------ */
/* Limber approximations (Sec. 2.2) and the non-linear correction (Sec. 3.2) */
/* ------------------------------------------------------------------------ */

/* Where the Limber approximation samples P: k[l][a] = (ell_l + 1/2) / chi_a at chi1 = chi2 =
 * chi_a (host [n_ell][n_chi], plan ell order). */
blast_status blast_plan_limber_k(const blast_plan *plan, double *k);

typedef struct {
    int32_t batch;
    int32_t p_dtype;          /* 0: P and P_sub are double, 1: float */
    const void *P;            /* device [batch][n_ell][n_chi]: P(k[l][a], chi_a, chi_a), plan ell order */
    const void *P_sub;        /* device, nullable: same layout, subtracted from P */
    int32_t n_g, n_s;         /* bins as in blast_cl_args */
    const double *K_chi;      /* device [batch][n_g + n_s][n_chi]: calligraphic kernels at chi_a */
    uint32_t types;           /* subset of the plan's types */
    int32_t n_ell_out;        /* 0: all plan multipoles */
    const int32_t *ell_idx;   /* host [n_ell_out], increasing indices into the plan's ell */
    int32_t order;            /* 1: Limber, 2: extended Limber (needs n_chi >= 5) */
    int32_t accumulate;       /* 0: C = C_limb, 1: C += C_limb */
    double *C;                /* device [batch][n_pairs][n_ell_out], pair order as blast_cl_forward */
} blast_limber_args;

/* Limber spectra on the plan's chi quadrature, in FP64:
 *   C_ij(l) = N_t(l) (pi/2) sum_a wchi_a f_t(k)/k^2 (P - P_sub)[l][a] / chi_a^2 E_ij(l, a),
 * k = (l+1/2)/chi_a; E = K_i K_j for order 1 and, for order 2 (the extended approximation),
 *   E = K_i K_j - nu^-2 sqrt(chi) [(chi^2/2 Kt_i'' + chi^3/6 Kt_i''') K_j + (i <-> j)],
 * nu = l + 1/2, Kt = K / sqrt(chi), with the derivatives of the degree-4 polynomial through
 * the 5 nearest chi nodes.  (The paper prints the bracket with a plus sign; the minus sign
 * of the underlying Bessel expansion gives the O(nu^-4) error it states.)  With P = the
 * non-linear and P_sub = the linear spectrum at the Limber points, and accumulate = 1 on
 * the output of blast_cl_forward for the linear spectrum, C becomes the corrected
 * C_lin + C_nl^limb - C_lin^limb of Sec. 3.2.  Asynchronous on `stream`.  Errors: INVALID
 * (shapes, types, order 2 with n_chi < 5), OOM, HIP. */
blast_status blast_cl_limber(blast_plan *plan, const blast_limber_args *args, void *stream);

/* Waits for the recorded events, writes the summed milliseconds of each stage
 * (host [4]) and the number of recorded calls, and clears the record. */
blast_status blast_plan_profile_read(blast_plan *plan, double *stage_ms, int64_t *calls);

#ifdef __cplusplus
}
#endif
#endif /* BLAST_HIP_H */
