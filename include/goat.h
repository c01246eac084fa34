/*
 * goat.h - C ABI of libgoat, the MI355X (gfx950) hot path of GOAT
 * ("Graph Matching via Optimal Transport", arXiv 2111.05366).
 *
 * Problem (Background, eqs. (QAP), (rQAP), (GM)): for n x n matrices A, B,
 * maximise f(P) = tr(A^T P B P^T) - equivalently minimise -tr(A P B^T P^T) -
 * over the Birkhoff polytope D of doubly stochastic matrices with the
 * Frank-Wolfe method of Alg. 3 (GOAT), whose direction step is entropic
 * optimal transport (Alg. 2, LOT), then project to a permutation with one
 * linear assignment.
 *
 * Conventions shared by every call
 *  - Matrices are row-major float32 n x n with a leading dimension ld >= n
 *    (in elements); a matrix buffer holds n*ld elements. Unless a call says
 *    "host", pointers are device pointers (HIP global memory).
 *  - Vectorised loads need ld % 4 == 0 and 16-byte aligned bases; other
 *    inputs are first repacked into the workspace (slower, still correct).
 *  - The caller owns every buffer; the library never frees caller memory.
 *    Scratch space is a caller-provided device workspace of at least
 *    goat_workspace_size(n, prec, symmetric) bytes, 256-byte aligned.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *    goat_grad, goat_sinkhorn and goat_linesearch are asynchronous on it and
 *    write scalar results to device memory; goat_solve is host-synchronous.
 *  - Return value: GOAT_OK (0) or a negative status. GOAT_EINVAL: null
 *    pointer, n < 1, ld < n, bad option. GOAT_ENOMEM: workspace too small.
 *    GOAT_EHIP: HIP runtime failure. GOAT_ENOTSUP: unsupported mode. The
 *    message of the last failure on the calling thread is goat_last_error().
 *    Non-convergence of an iteration is not an error; it is reported in
 *    the outputs.
 *
 * Entry points
 *  - one Frank-Wolfe iteration's pieces: goat_grad (Alg. 3 step 1; or
 *    goat_pack once and goat_grad_packed per gradient),
 *    goat_sinkhorn (LOT direction, Alg. 2), goat_linesearch (step 3);
 *  - whole solves: goat_solve, goat_run_begin/steps/finish/gradient/free,
 *    goat_solve_seeded (seeds, unequal sizes), goat_random_init and
 *    goat_solve_restarts (random starts), goat_batch_* and goat_tune (many
 *    pairs and starts in one launch);
 *  - the final projection: goat_lap_max (host), goat_lap_device (device),
 *    goat_score; soft matching: goat_nominate;
 *  - the learned Sinkhorn warm start: goat_mlp_*;
 *  - sizes, options, errors, timing: goat_workspace_size,
 *    goat_default_options, goat_version, goat_last_error,
 *    goat_profile_enable/read.
 */
#ifndef GOAT_H
#define GOAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GOAT_OK        0
#define GOAT_EINVAL   -1
#define GOAT_EHIP     -2
#define GOAT_ENOMEM   -3
#define GOAT_ENOTSUP  -4

/* Arithmetic of the gradient products (all accumulate in float32).
 *  FP32   : float32 operands on the fp32 matrix cores.
 *  BF16X2 : A, B rounded to bf16 (exact for 0/1 adjacency), the P-side
 *           operand split into bf16 hi + lo parts: 2 bf16 products.
 *  BF16X3 : A, B and the P-side operand all split hi + lo; the lo*lo term
 *           is dropped: 3 bf16 products (weighted graphs).
 *  FP8    : A, B in FP8 E4M3 (exact for 0/1 adjacency), the P-side operand
 *           split into three scaled E4M3 terms: 3 fp8 products (see
 *           goat_grad).                                                */
#define GOAT_PREC_FP32    0
#define GOAT_PREC_BF16X2  1
#define GOAT_PREC_BF16X3  2
#define GOAT_PREC_FP8     3

/* Sinkhorn starting potentials. */
#define GOAT_INIT_COLD  0   /* g = 0                                   */
#define GOAT_INIT_G     1   /* start from the caller's g               */
#define GOAT_INIT_MLP   2   /* g from the warm-start network (see the
                               learned warm start below)               */

/* Library version as 10000*major + 100*minor + patch. */
int goat_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char* goat_last_error(void);

/* Bytes of device workspace that every call below needs at size n with
 * the given precision and symmetry flag. */
size_t goat_workspace_size(int n, int prec, int symmetric);

/*
 * goat_grad - gradient of the relaxed objective (Alg. 3 step 1):
 *     G = A P B^T + A^T P B.
 * A, B, P: inputs (lda = ldb = ld, ldp), G: output (ldg). With
 * symmetric != 0 the caller promises A = A^T and B = B^T and the library
 * evaluates G = 2 A P B (two products instead of four). prec selects the
 * arithmetic (GOAT_PREC_*). BF16X2 requires A and B exactly representable
 * in bf16 (e.g. 0/1 adjacency); it is the caller's promise. FP8 requires A
 * and B exactly representable in FP8 E4M3 (0/1 adjacency, small integers);
 * P and the intermediate product enter as three E4M3 terms each (term t of
 * x is E4M3 of the residual times 2^(s + 4t), s from max|x|), so the
 * products run on the FP8 matrix cores with FP32 accumulation and about 12
 * significant bits per operand element.
 */
int goat_grad(int n, const float* A, const float* B, int ld,
              const float* P, int ldp, float* G, int ldg,
              int prec, int symmetric,
              void* ws, size_t ws_bytes, void* stream);

/*
 * goat_pack / goat_grad_packed - goat_grad in two parts, for callers that
 * take many gradients of one pair: goat_pack converts A and B once into the
 * matrix-core operands of `prec` (fp32, bf16, bf16 hi + lo planes or FP8
 * E4M3; [X; X^T] stacked when symmetric = 0), zero padded, into the
 * workspace (goat_workspace_size(n, prec, symmetric) bytes); every
 * goat_grad_packed call with the same workspace, n, prec and symmetric then
 * computes G = grad f(P) (Alg. 3 step 1) from them. The packed operands stay
 * valid until the workspace is used by another call; goat_grad packs into
 * the same place, so goat_grad_packed after goat_grad reuses its operands.
 * Results are those of goat_grad, bit for bit. Asynchronous on `stream`.
 */
int goat_pack(int n, const float* A, const float* B, int ld, int prec, int symmetric,
              void* ws, size_t ws_bytes, void* stream);
int goat_grad_packed(int n, const float* P, int ldp, float* G, int ldg, int prec, int symmetric,
                     void* ws, size_t ws_bytes, void* stream);

/*
 * goat_sinkhorn - LOT direction (Alg. 2 with the cost negated, as the
 * Methods section prescribes for the maximisation in Alg. 3 step 2): the
 * entropic maximiser of tr(Q^T G) over D,
 *     Q_ij = exp((G_ij + f_i + g_j) / eps),
 * found by log-domain Sinkhorn-Knopp scaling (Sinkhorn distance, eq. (5)).
 * Each iteration sets f from the row sums, then g from the column sums.
 * Stop: after a column update, the largest row-marginal error
 * max_i |sum_j Q_ij - 1| of the current plan is <= tol (checked from the
 * second iteration on), or max_iter column updates have run.
 *
 *  G        n x n input (ldg).
 *  eps_dev  device float: the eps to use; NULL = eps_rel * max|G|
 *           computed on the device. If the resulting eps is 0, Q = J.
 *  f, g     device float[n]: final potentials (natural units). With
 *           init == GOAT_INIT_G, g is read first as the starting point.
 *  init     GOAT_INIT_COLD (g = 0), GOAT_INIT_G (the caller's g) or
 *           GOAT_INIT_MLP: g = eps * network(column features of G / eps)
 *           with the parameters at mlp_params (device float, the packed
 *           layout of goat_mlp_param_count; n <= 20480). Every start
 *           leads to the same fixed point; only the sweeps to reach it
 *           differ.
 *  mlp_params  device parameters for GOAT_INIT_MLP, else ignored (NULL).
 *  Q        n x n output (ldq), or NULL to skip forming it.
 *  iters_dev, err_dev, eps_out  device int / float / float outputs (each
 *           may be NULL): column updates run, max_i |sum_j Q_ij - 1| of the
 *           returned plan, and the eps used.
 * The call is asynchronous; convergence is decided on the device. Every
 * sweep after the first uses compensated (two-float) potentials, so that
 * marginal errors near 1e-6 are resolved. G is copied into the workspace
 * (one extra read and write of G) when ldg is not a multiple of 4, G is not
 * 16-byte aligned, or ldg is not a multiple of 64 and max_iter >= 8.
 */
int goat_sinkhorn(int n, const float* G, int ldg,
                  const float* eps_dev, float eps_rel,
                  float* f, float* g, int init, const float* mlp_params,
                  int max_iter, float tol,
                  float* Q, int ldq,
                  int* iters_dev, float* err_dev, float* eps_out,
                  void* ws, size_t ws_bytes, void* stream);

/*
 * goat_sinkhorn_noalloc - goat_sinkhorn without a workspace, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc). Same arguments, kernels
 * and results as goat_sinkhorn (bit for bit); the solver's state lives in a
 * static device array of goat_sinkhorn_noalloc_scratch_bytes() (64 MiB) that
 * every GPU the library runs on holds until the process ends. The call
 * allocates nothing and never takes profiler events.
 *  n        1 <= n <= goat_sinkhorn_noalloc_max_n() (about 16,000 nodes).
 *  G        16-byte aligned, ldg a multiple of 4, and of 64 when
 *           max_iter >= 8 (G is never repacked).
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (different streams or host threads) race and give wrong results; calls
 * ordered on one stream are safe. Each call initialises the state it reads.
 * Status: as goat_sinkhorn; GOAT_EINVAL also for n above the limit or a G
 * that would need repacking.
 */
size_t goat_sinkhorn_noalloc_scratch_bytes(void);
int    goat_sinkhorn_noalloc_max_n(void);
int    goat_sinkhorn_noalloc(int n, const float* G, int ldg,
                             const float* eps_dev, float eps_rel,
                             float* f, float* g, int init, const float* mlp_params,
                             int max_iter, float tol,
                             float* Q, int ldq,
                             int* iters_dev, float* err_dev, float* eps_out,
                             void* stream);

/*
 * goat_linesearch - exact step of Alg. 3 step 3. With D = Q - P the
 * objective is the quadratic f(P + tD) = fP + b t + a t^2 where
 *     fP = <P,GP>/2, fQ = <Q,GQ>/2, c = <Q,GP>, a = fP + fQ - c, b = c - 2 fP
 * (GP = grad f(P), GQ = grad f(Q)); t maximises it over [0, 1] (the
 * paper's alpha is 1 - t). All traces accumulate in float64.
 * out_dev: device double[8] = {fP, fQ, c, a, b, t, ||Q-P||_F^2, 0}.
 */
int goat_linesearch(int n, const float* P, const float* Q,
                    const float* GP, const float* GQ, int ld,
                    double* out_dev,
                    void* ws, size_t ws_bytes, void* stream);

/* Options of goat_solve; goat_default_options() fills the defaults. */
typedef struct goat_options {
    float eps_rel;        /* eps = eps_rel * max|grad f(P)| per FW iteration (0.03) */
    float sk_tol;         /* Sinkhorn row-marginal tolerance (1e-6)                 */
    int   sk_max;         /* Sinkhorn iteration cap (1000)                          */
    int   fw_max;         /* Frank-Wolfe iteration cap (30)                         */
    float fw_tol;         /* stop when t ||Q-P||_F / sqrt(n) < fw_tol; 0 = off      */
    int   prec;           /* GOAT_PREC_*                                            */
    int   symmetric;      /* 1: A = A^T and B = B^T                                 */
    int   proj;           /* 0: final LAP on P_final; 1: on grad f(P_final)         */
    int   warm;           /* Sinkhorn start: 0 cold; 1 the previous iteration's
                             column potentials; 2 the warm-start network each
                             iteration; 3 the network first, then as 1            */
    int   stop_on_stall;  /* 1: stop when t == 0 (default); 0: run fw_max iterations */
    int   check_every;    /* Sinkhorn convergence flag polled every k iterations (16) */
    int   lap;            /* final assignment: 0 host Jonker-Volgenant on float64
                             scores (default); 1 device auction on the quantised
                             scores (goat_lap_device; in a batch one workgroup
                             per problem); its errors are returned            */
    int   sk_g24;         /* 1: the Sinkhorn sweeps and Q read a 24-bit fixed-point
                             copy of grad f(P), q = rint(G (2^23-1) / max|G|), made
                             once per FW iteration: 3 bytes per entry instead of 4,
                             G eps^-1 within max|G|/eps 2^-24 of the float value
                             (mixed precisions only; 0: float G, the default)  */
    int   reserved[3];
    const float* mlp_params; /* device float[goat_mlp_param_count()] (warm 2, 3) */
} goat_options;

/* Per-iteration record of goat_solve (host memory). */
typedef struct goat_iter_record {
    double fP, fQ, c, a, b, t, dist2;  /* line-search scalars of this iteration */
    float  eps;                        /* eps used by Sinkhorn                  */
    float  sk_err;                     /* row-marginal error of Q               */
    int    sk_iters;                   /* Sinkhorn column updates               */
    int    pad;
} goat_iter_record;

typedef struct goat_stats {
    int    fw_iters;       /* Frank-Wolfe iterations run                      */
    int    sk_iters_total; /* Sinkhorn iterations summed over FW iterations   */
    int    sk_capped;      /* FW iterations whose Sinkhorn hit sk_max         */
    int    lap_device;     /* 1: the final assignment ran on the device       */
    double f_final;        /* f(P_final) = tr(A^T P B P^T)                    */
    double score;          /* tr(A^T Pi B Pi^T) of the returned permutation   */
    double ms_loop;        /* device time of the FW loop (HIP events)         */
    double ms_lap;         /* wall time of the final assignment               */
    double ms_total;       /* wall time of the call                           */
} goat_stats;

void goat_default_options(goat_options* opt);

/*
 * goat_solve - Alg. 3 end to end for one pair: P0 (NULL = barycenter
 * J = 11^T/n, the initialisation of Alg. 1 and Alg. 3; else an n x n
 * doubly stochastic device matrix with leading dimension ld), Frank-Wolfe
 * iterations (gradient, LOT direction, exact step, update), then
 * perm = argmax over permutations of <Pi, P_final> (or of
 * <Pi, grad f(P_final)> with opt->proj = 1) by a host linear assignment
 * (opt->lap = 0) or the device auction (opt->lap = 1).
 *  perm_host  host int32[n]: perm[i] = j matches A-node i to B-node j.
 *  stats_host host goat_stats (may be NULL).
 *  hist_host  host goat_iter_record[hist_cap] (may be NULL).
 *  P_out      device n x n (ld) final relaxed P, or NULL.
 * Host-synchronous on `stream`. A or B holding a NaN or an infinity is
 * refused with GOAT_EINVAL before any iteration (one device pass over each).
 */
int goat_solve(int n, const float* A, const float* B, int ld,
               const float* P0, const goat_options* opt,
               int32_t* perm_host, goat_stats* stats_host,
               goat_iter_record* hist_host, int hist_cap,
               float* P_out,
               void* ws, size_t ws_bytes, void* stream);

/*
 * Stepwise form of goat_solve, for callers that time or inspect a fixed
 * number of Frank-Wolfe iterations (Alg. 3 loop body):
 *  goat_run_begin   packs A and B, sets P0 (NULL = barycenter) and computes
 *                   grad f(P0); the workspace must stay untouched until
 *                   goat_run_free. *run receives a host handle.
 *  goat_run_steps   runs up to k iterations (fewer once stopped by a stall
 *                   or fw_tol when those stops are enabled); hist_host gets
 *                   one record per iteration run, *done_out their number.
 *                   opt->fw_max does not limit this call.
 *  goat_run_finish  final assignment on P (or grad f(P)), the score of the
 *                   permutation, optional copy of P to P_out (ldp). With
 *                   opt->lap = 1 the device assignment may take G_Q and the
 *                   packed operands as its workspace: goat_run_steps then
 *                   returns GOAT_EINVAL (finish, gradient and free still
 *                   work).
 *  goat_run_free    releases the handle (host memory, events).
 *  goat_run_gradient copies the current grad f(P) out (device to device).
 * All host-synchronous on the stream given to goat_run_begin.
 */
typedef struct goat_run goat_run;
int  goat_run_begin(int n, const float* A, const float* B, int ld,
                    const float* P0, const goat_options* opt,
                    void* ws, size_t ws_bytes, void* stream, goat_run** run);
int  goat_run_steps(goat_run* run, int k, goat_iter_record* hist_host,
                    int hist_cap, int* done_out);
int  goat_run_finish(goat_run* run, int32_t* perm_host, goat_stats* stats_host,
                     float* P_out, int ldp);
void goat_run_free(goat_run* run);
/* Copy of the run's current gradient grad f(P) (n x n, ldg) into G_out. */
int  goat_run_gradient(goat_run* run, float* G_out, int ldg);
/* Copy of the last iteration's LOT direction Q (Alg. 3 step 2; n x n, ldq)
 * into Q_out. GOAT_EINVAL before the first iteration or after a device
 * assignment that reused the run's buffers. */
int  goat_run_direction(goat_run* run, float* Q_out, int ldq);
/* Sinkhorn cap and tolerance for the following goat_run_steps calls (a
 * schedule per iteration, e.g. a fixed sweep count to replay another run).
 * GOAT_EINVAL for sk_max < 1 or a negative or non-finite tolerance. */
int  goat_run_set_sinkhorn(goat_run* run, int sk_max, float sk_tol);

/*
 * Kernel timing hook (measurement only). which = 0: Sinkhorn row sweep;
 * which = 1: gradient product. With stride > 0, every stride-th such launch
 * made by the calling thread is timed (at most 8192 samples are kept): a
 * row sweep by events that its launch itself records at the kernel's start
 * and end (hipExtLaunchKernel), a product (its matrix-core launches) by
 * events recorded on its stream before and after.
 * goat_profile_read waits for the sampled launches, returns their summed
 * duration (ms) and count, and clears the samples. stride = 0 disables.
 */
int goat_profile_enable(int which, int stride);
int goat_profile_read(int which, double* ms_total, long long* count);

/*
 * Learned Sinkhorn warm start (not in the paper; the network replaces the
 * cold start g = 0 of Alg. 2's Sinkhorn solve, whose fixed point it does not
 * change). Features of column j of X = G / eps: mean_i, max_i, population
 * std_i and LSE_i x_ij - log n, each centred over j; network
 * 4 -> 128 -> 128 -> 1 with ReLU, float32, predicting g_j / eps (centred).
 * Parameters: device float[goat_mlp_param_count()] packed W1[128][4], b1,
 * W2[128][128], b2, W3[128], b3.
 *  goat_mlp_features  F: device float[n][4]; eps_dev: device float; the
 *                     workspace is the one of goat_workspace_size(n, ...)
 *                     (G is repacked into it when ld % 4 != 0 or it is
 *                     not 16-byte aligned); n <= 20480.
 *  goat_mlp_forward   y[N] = network(F[N][4]).
 *  goat_mlp_backward  grad = d/dparams of (1/N) sum (y - target)^2 and the
 *                     loss (loss_dev may be NULL); workspace of
 *                     goat_mlp_workspace_size(N) bytes; deterministic.
 *  goat_mlp_adam      one Adam step (beta 0.9 / 0.999, eps 1e-8, bias
 *                     corrected; step counts from 1) on params, m, v.
 */
int    goat_mlp_param_count(void);
size_t goat_mlp_workspace_size(int n_samples);
int    goat_mlp_features(int n, const float* G, int ldg, const float* eps_dev,
                         float* F, void* ws, size_t ws_bytes, void* stream);
int    goat_mlp_forward(int N, const float* F, const float* params, float* y,
                        void* stream);
int    goat_mlp_backward(int N, const float* F, const float* target,
                         const float* params, float* grad, float* loss_dev,
                         void* ws, size_t ws_bytes, void* stream);
int    goat_mlp_adam(const float* grad, float* params, float* m, float* v,
                     int step, float lr, void* stream);

/*
 * goat_lap_max - host linear assignment (Alg. 3 return line; Alg. 1 step 2
 * uses the same problem): perm maximising sum_i M[i*ld + perm[i]] over
 * permutations, for a host float64 matrix M. Jonker-Volgenant shortest
 * augmenting paths from a greedy start; deterministic tie-breaking (lowest
 * column index among equal path lengths). O(n^3) worst case.
 */
int goat_lap_max(int n, const double* M_host, int ld, int32_t* perm_host);

/*
 * goat_lap_device - the same projection on the device for a device float
 * matrix M (n x n, leading dimension ld): Bertsekas' auction with epsilon
 * scaling on integer scores. Unassigned rows bid in parallel rounds; when
 * few are left, or a batch of rounds assigns few rows, one workgroup takes
 * the bids in sequence; each phase keeps the pairs that stay optimal to
 * within the new epsilon. A bid in sequence first tries the row's list of
 * 64 candidate columns, kept from its last scan with a bound on every
 * other column's value (prices only rise, so the bound holds); only when
 * the list cannot decide the bid is the row scanned again. With 2^(e-1) <= max|M| < 2^e,
 * R = min(40, 55 - ceil(log2(n+1))) and s = R - 1 - e, the scores are
 * c_ij = rint(M_ij * 2^s) - min_kl rint(M_kl * 2^s) (round half to even;
 * 0 <= c <= 2^R), and perm maximises sum_i c[i][perm i] exactly; on M
 * itself it is within n * 2^-s of the optimum. Equal bids go to the lowest
 * row, so the result is deterministic. All-equal c gives the identity.
 *  perm_dev   device int32[n] (row i -> column perm_dev[i]).
 *  ws         device workspace of goat_lap_device_workspace_size(n) bytes
 *             (about 8 n^2: the scaled scores are precomputed once as int64
 *             and every scan reads them), or at least
 *             goat_lap_device_workspace_min(n) bytes (about 820 n, most of
 *             it the candidate lists: every scan converts M again). Both
 *             give the same result.
 *  max_rounds cap on parallel rounds plus tail bids over all phases
 *             (<= 0: 20,000,000).
 *  stats      host goat_lap_stats (may be NULL).
 * Host-synchronous on `stream` (it polls a device counter between batches
 * of rounds).
 * Status: GOAT_EINVAL for n < 1, n >= 2^20 - 1, ld < n, null pointers or a
 * non-finite entry; GOAT_ENOMEM for a short workspace; GOAT_ENOTSUP when
 * the round cap is reached or a bid would exceed 2^62 (the host solver,
 * goat_lap_max, has neither limit).
 */
typedef struct goat_lap_stats {
    long long rounds;           /* parallel bidding rounds that ran         */
    long long rounds_launched;  /* parallel rounds enqueued + sequential budgets */
    long long tail_bids;        /* bids taken in sequence                   */
    int phases;                 /* epsilon phases                           */
    int shift;                  /* s above                                  */
    int resolution_bits;        /* R above                                  */
    int list_bids;              /* of the tail bids, those decided by the
                                   row's candidate list without a row scan */
    int skipped_phases;         /* of the phases, those passed over without
                                   a launch: an idle phase's filter kept every
                                   pair, and these later phases' epsilon is
                                   at least its largest slack            */
} goat_lap_stats;
size_t goat_lap_device_workspace_size(int n);
size_t goat_lap_device_workspace_min(int n);
int goat_lap_device(int n, const float* M, int ld, int32_t* perm_dev,
                    void* ws, size_t ws_bytes, long long max_rounds,
                    goat_lap_stats* stats, void* stream);

/*
 * goat_score - tr(A^T Pi B Pi^T) = sum_ij A_ij B_{perm i, perm j} for a
 * device int32 permutation (entries outside [0, n) are clamped into range;
 * the result is meaningful only for a permutation), accumulated in float64
 * (the (QAP) objective at a permutation; graph matching minimises its
 * negation, eq. (GM)). out_dev: device double.
 */
int goat_score(int n, const float* A, const float* B, int ld,
               const int32_t* perm_dev, double* out_dev,
               void* ws, size_t ws_bytes, void* stream);

/*
 * goat_nominate - soft matching (vertex nomination; the Discussion names it
 * as a use of the relaxed solution): for each row i of the device float
 * matrix P (rows x cols, row-major, leading dimension ldp >= cols; the
 * final iterate of goat_run_finish / goat_batch_get_P, or a Sinkhorn
 * direction Q) the k columns with the largest P[i, j], best first; equal
 * scores rank by increasing column. Writes idx_dev[i*k + r] (device int32,
 * rows*k entries) and, unless val_dev is NULL, val_dev[i*k + r] = the score
 * (device float). NaN scores are never nominated; a row with fewer than k
 * other scores ends in -1 entries. Reads P once; no workspace; asynchronous
 * on `stream`.
 * Status: GOAT_EINVAL for rows or cols < 1, k outside [1, min(cols,
 * GOAT_NOMINATE_KMAX)], ldp < cols, null P or idx_dev.
 */
#define GOAT_NOMINATE_KMAX 32
int goat_nominate(int rows, int cols, const float* P, int ldp, int k,
                  int32_t* idx_dev, float* val_dev, void* stream);

/* ------------------------------------------------------------------------
 * Seeds and graphs of different sizes
 * ---------------------------------------------------------------------- */

/*
 * goat_solve_seeded - GOAT with seeds and unequal sizes: Fishkind et al.'s
 * modification of FAQ (cited by the paper for seeded graph matching and
 * applied there to GOAT) on Alg. 3. Seed i of A is matched to seed i of B;
 * the remaining vertices follow in increasing order; the smaller graph is
 * padded with isolated dummy vertices to n = max(nA, nB), after recentring
 * both graphs to 2X - J when pad = 1 ("adopted" padding, for 0/1 graphs;
 * pad = 0: "naive"). With Pi = diag(I_m, P) the objective is
 * tr(A11^T B11) + <C, P> + tr(A22^T P B22 P^T), C = A21 B21^T + A12^T B12, so
 * Alg. 3 runs on the non-seed block with C added to every gradient (C on the
 * fp32 matrix cores) and the exact step extended by the linear term.
 *  A: nA x nA (lda), B: nB x nB (ldb), device.
 *  seeds_A, seeds_B: host int32[m], distinct vertices of A and of B.
 *  perm_host: host int32[nA]: the B vertex matched to each A vertex, -1 when
 *           it is matched to a dummy (nA > nB).
 *  stats_host: as goat_solve for the non-seed block (f_final excludes the
 *           constant tr(A11^T B11)); score = tr(A'^T Pi B' Pi^T) of the
 *           arranged (recentred, padded) graphs. hist_host: as goat_solve.
 *  ws: goat_seeded_workspace_size(nA, nB, m, opt->prec, opt->symmetric) bytes.
 * Status: GOAT_EINVAL for bad sizes, seeds (repeated or out of range), pad
 * or options; GOAT_ENOMEM; GOAT_EHIP. Host-synchronous, like goat_solve.
 */
size_t goat_seeded_workspace_size(int nA, int nB, int m, int prec, int symmetric);
int goat_solve_seeded(int nA, const float* A, int lda, int nB, const float* B, int ldb, int m,
                      const int32_t* seeds_A, const int32_t* seeds_B, int pad,
                      const goat_options* opt, int32_t* perm_host, goat_stats* stats_host,
                      goat_iter_record* hist_host, int hist_cap,
                      void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Random starts (GOAT section, random initialisations)
 * ---------------------------------------------------------------------- */

/*
 * goat_random_init - P0 = (J + K) / 2, where J = 1 1^T / n is the barycenter
 * and K = diag(r) U diag(c) is the Sinkhorn-Knopp scaling of a positive n x n
 * matrix U to a doubly stochastic one. Sweeps run until
 * max_i |(K 1)_i - 1| <= tol (checked from the second sweep) or max_iter
 * sweeps; float32 on the device. For n <= GOAT_BATCH_NMAX one workgroup
 * alternates r = 1 / (U c), c = 1 / (U^T r) from c = 1 in LDS (no
 * workspace). Above, K is the entropic plan of the cost ln U at eps = 1,
 * computed by goat_sinkhorn's sweeps (column potentials from 0) on ln U kept
 * in the workspace.
 *  U        device n x n (ldu >= n), entries > 0 (e.g. U(0,1) draws).
 *  P        device n x n output (ldp >= n).
 *  iters_dev, err_dev  device int / float (may be NULL): sweeps run and the
 *           final row-sum error of K.
 *  ws       device workspace of goat_random_init_workspace_size(n) bytes
 *           (0, and ws may be NULL, for n <= GOAT_BATCH_NMAX; about 4 n^2
 *           above).
 * Asynchronous on `stream`.
 * Status: GOAT_EINVAL for n < 1, bad ld, null U or P, tol < 0 or not finite,
 * max_iter < 1; GOAT_ENOMEM for a short workspace. Non-positive entries of U
 * are not checked (the scaling then produces inf or nan).
 */
#define GOAT_BATCH_NMAX 1024
size_t goat_random_init_workspace_size(int n);
int goat_random_init(int n, const float* U, int ldu, float* P, int ldp, float tol, int max_iter,
                     int* iters_dev, float* err_dev, void* ws, size_t ws_bytes, void* stream);

/*
 * goat_solve_restarts - GOAT from several random starts for one pair of any
 * size (GOAT section, random initialisations): restart r starts at
 * P0 = (J + SK(U_r)) / 2 (goat_random_init, tolerance 1e-6, at most 1000
 * sweeps) with U_r the n x n matrix at U + r * n * ldu, and runs goat_solve
 * with opt; the permutation with the largest tr(A^T Pi B Pi^T) is kept, ties
 * to the lowest r.
 *  U            device, restarts stacked n x n positive draws (ldu >= n).
 *  perm_host    host int32[n]: the kept permutation.
 *  scores_host  host double[restarts] (may be NULL): each restart's score.
 *  best_host    host int (may be NULL): the kept restart.
 *  stats_host   host goat_stats (may be NULL): the kept restart's stats.
 *  ws           goat_solve_restarts_workspace_size(n, ld, prec, symmetric)
 *               bytes: goat_solve's workspace, P0 (n x ld) and the random
 *               start's.
 * Host-synchronous, like goat_solve. Status: GOAT_EINVAL for bad sizes,
 * pointers, restarts < 1 or options; GOAT_ENOMEM; goat_solve's errors.
 */
size_t goat_solve_restarts_workspace_size(int n, int ld, int prec, int symmetric);
int goat_solve_restarts(int n, const float* A, const float* B, int ld, const float* U, int ldu,
                        int restarts, const goat_options* opt, int32_t* perm_host,
                        double* scores_host, int* best_host, goat_stats* stats_host,
                        void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Batched solve: many graph pairs of uneven size, several starts each
 * ---------------------------------------------------------------------- */

/* One graph pair of a batch. */
typedef struct goat_pair {
    int n;               /* nodes, 1 <= n <= GOAT_BATCH_NMAX                      */
    int ld;              /* leading dimension of A, B, U (>= n)                   */
    const float* A;      /* device n x n                                          */
    const float* B;      /* device n x n                                          */
    const float* U;      /* device positive draws for the random starts: restart r
                            uses the n x n matrix at U + r * n * ld and starts at
                            (J + SK(U_r)) / 2 (see goat_random_init); NULL: every
                            restart starts at J                                   */
} goat_pair;

typedef struct goat_batch goat_batch;

typedef struct goat_batch_stats {
    int    problems;       /* npairs * restarts                                 */
    int    fw_iters_total; /* FW iterations summed over problems                */
    long long sk_iters_total; /* Sinkhorn iterations summed over problems       */
    int    sk_capped;      /* (problem, FW iteration)s whose Sinkhorn hit sk_max */
    int    launches;       /* kernels in the graph (one per size bucket + packing) */
    double ms_graph;       /* device time of the graph launch (HIP events)      */
    double ms_lap;         /* host time of all final assignments                */
    double ms_total;       /* wall time of goat_batch_results                   */
    long long lap_bids;    /* device assignments (opt.lap = 1): bids summed over
                              problems; 0 with the host solver                 */
} goat_batch_stats;

/*
 * goat_batch_create - plan a batch: npairs pairs x restarts starts, each a
 * full GOAT solve (Alg. 3: Frank-Wolfe with the LOT direction, exact step,
 * final assignment) with the options of opt (eps_rel, sk_tol, sk_max, fw_max,
 * fw_tol, symmetric, proj, stop_on_stall, warm 0 or 1; prec must be
 * GOAT_PREC_FP32). One workgroup runs one (pair, start) problem from its
 * start to its last FW iteration inside a single persistent kernel; problems
 * are grouped into size buckets, each bucket one kernel with its autotuned
 * shape (goat_tune), all captured in one HIP graph. The pair descriptors are
 * copied; A, B, U must stay valid and unchanged until goat_batch_destroy.
 *  ws, ws_bytes  device workspace of at least goat_batch_workspace_size bytes,
 *           owned by the caller, in use until goat_batch_destroy.
 * Status: GOAT_EINVAL (bad pair, restarts < 1, options, or a pair whose A
 * or B holds a NaN or an infinity, checked on the device at creation),
 * GOAT_ENOTSUP (prec != FP32, warm > 1), GOAT_ENOMEM (workspace too
 * small), GOAT_EHIP.
 */
int goat_batch_workspace_size(const goat_pair* pairs, int npairs, int restarts,
                              const goat_options* opt, size_t* bytes);
int goat_batch_create(const goat_pair* pairs, int npairs, int restarts,
                      const goat_options* opt, void* ws, size_t ws_bytes,
                      goat_batch** out);
/* Launch the whole batch (one graph launch), stream-ordered on stream. */
int goat_batch_launch(goat_batch* b, void* stream);
/*
 * goat_batch_results - wait for the launch, then the final assignments (on
 * the host, one LAP per problem, problems in parallel; with opt->lap = 1 on
 * the device, one workgroup per problem, the quantised auction of
 * goat_lap_device with a budget of 4,000,000 bids per problem), scores
 * tr(A^T Pi B Pi^T) on the device, and per pair the start with the largest
 * score (ties to the lowest start index). A device assignment that spends
 * its budget returns GOAT_ENOTSUP, one that meets a non-finite score
 * GOAT_EINVAL.
 *  perm_host   int32[sum_p n_p]: kept permutation of each pair, concatenated
 *              in pair order (may be NULL).
 *  score_host  double[npairs] (may be NULL); best_host int[npairs] (may be NULL).
 *  all_score_host double[npairs * restarts], pair-major (may be NULL).
 *  hist_host   goat_iter_record[npairs * restarts * hist_cap], problem
 *              (pair-major) then FW iteration; records past a problem's last
 *              iteration are zeroed (may be NULL).
 *  fw_iters_host int[npairs * restarts] (may be NULL).
 */
int goat_batch_results(goat_batch* b, int32_t* perm_host, double* score_host, int* best_host,
                       double* all_score_host, goat_iter_record* hist_host, int hist_cap,
                       int* fw_iters_host, goat_batch_stats* stats_host);
/* Copy the final P (proj = 0) of problem (pair, restart) to a device n x n
 * matrix out (ld >= n), stream-ordered. */
int goat_batch_get_P(goat_batch* b, int pair, int restart, float* out, int ld, void* stream);
void goat_batch_destroy(goat_batch* b);

/*
 * goat_tune - autotune the batched kernel's shape (lanes per Sinkhorn row)
 * for every size bucket up to n_max on the current device: each candidate
 * runs a synthetic batch of the bucket's largest size and the fastest is
 * kept in a per-device table that later goat_batch_create calls read
 * (untuned buckets use a fixed default). reps >= 1 timed launches each.
 * goat_tune_get reports the shape used for size n: lanes per row (16, 32 or
 * 64) and waves per workgroup.
 */
int goat_tune(int n_max, int reps, void* stream);
int goat_tune_get(int n, int* lanes_per_row, int* waves);

#ifdef __cplusplus
}
#endif

#endif /* GOAT_H */
