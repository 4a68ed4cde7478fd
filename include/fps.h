/*
 * fps.h -- C ABI of libfps, the MI355X (gfx950) implementation of the
 * filtered Paterson-Stockmeyer (PS) evaluation of a matrix power series
 *
 *     F(Z) = sum_{k=0..m} c_k Z^k          (paper eqs. 1 and 8)
 *
 * on a sparse n x n matrix Z, following "A filtering technique for the matrix
 * power series being near-sparse" (arXiv 2208.05683), Section 3 and
 * Algorithm 2, with a fixed entry threshold tau (the simple filter of
 * Section 3.1.1) in place of the adaptive filter of Algorithm 1.
 *
 * Computation (all on the GPU, all in IEEE binary64):
 *   N = m+1, q = s, b = ceil(N/q), g = [N - q(b-1) == 1]          (eq. 6)
 *   P_1 = Z, P_{j+1} = D_tau(Z (x) P_j)   for j < q  (or < m if b == 1)  (eq. 11)
 *   Bhat_i = sum_{j<q} c_{iq+j} P_j  with P_0 = I, not filtered        (eq. 13)
 *   S_0 = Bhat_{b-1};  if g == 1: S_1 = Bhat_{b-2} + c_{(b-1)q} P_q,
 *                                 with no product and no filter         (eq. 14)
 *   S_i = D_tau(Bhat_{b-1-i} + P_q (x) S_{i-1})                         (eq. 14)
 *   F = S_{b-1}
 * where D_tau drops x iff x == 0 or |x| < tau, and (x) is the row-wise
 * (Gustavson) product accumulating A_rk * B_k,: over ascending k with one
 * fused multiply-add per term from +0; Bhat and the g = 1 sum accumulate
 * c_j P_j over ascending j with fused multiply-adds from +0 (terms with
 * c_j == 0 skipped); a Horner step adds the block with one addition,
 * x = bhat + product.  With these conventions results are reproducible
 * bit for bit, independent of launch configuration.
 *
 * Conventions for every entry point:
 *   - Matrices are square with 1 <= n <= FPS_MAX_N (a term row is
 *     addressed with 32-bit byte offsets).
 *   - CSR views hold DEVICE pointers: row_ptr int64[n+1] with row_ptr[0] = 0,
 *     col int32[nnz] strictly increasing within each row, val double[nnz]
 *     finite.  Views are borrowed: the library never frees them.
 *   - Streams are hipStream_t values (NULL = the default stream).  Work is
 *     ordered on the stream passed in.
 *   - Functions return an fps_status; nothing throws across the ABI and
 *     nothing aborts.  fps_last_error() gives a thread-local message for the
 *     last failure on the calling thread.  Asynchronous device faults are
 *     reported by the next call that synchronises.
 *   - A plan or matrix handle must not be used from two host threads at once.
 */
#ifndef FPS_H
#define FPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FPS_ABI_VERSION 2

typedef int32_t fps_status;
#define FPS_OK 0
#define FPS_ERR_INVALID_ARG 1   /* bad scalar argument or null pointer */
#define FPS_ERR_BAD_CSR 2       /* input matrix fails validation */
#define FPS_ERR_OUT_OF_MEMORY 3 /* device allocation failed */
#define FPS_ERR_HIP 4           /* a HIP runtime call or kernel failed */
#define FPS_ERR_CAPACITY 5      /* a size limit of the library was exceeded */
#define FPS_ERR_NOT_READY 6     /* result requested before any evaluation */

/* largest PS block size s accepted (the g = 1 sum has s+1 terms) */
#define FPS_MAX_S 31
/* Largest supported matrix dimension n. */
#define FPS_MAX_N 268435456
/* number of per-stage records kept in fps_stats */
#define FPS_MAX_STAGES 96

/* plan flags */
#define FPS_FLAG_NO_SKIP 0x1ull      /* disable the exact bound-based row skip */
#define FPS_FLAG_FORCE_GLOBAL 0x2ull /* route every row through the global-memory kernel */
#define FPS_FLAG_TIMING 0x4ull       /* record HIP events around the numeric kernels of every stage (the
                                        shared-memory kernel and the fallback tiers after it, or the dense
                                        path) of the first evaluation after a statistics query and every
                                        8th one after it */
#define FPS_FLAG_NO_VALIDATE 0x8ull  /* skip the device-side CSR check of Z at plan time */
#define FPS_FLAG_SYNC_SIZES 0x10ull  /* size every stage from a host read (no learned capacities) */
#define FPS_FLAG_DROP_STATS 0x20ull  /* fixed threshold: per filtered product, count the entries that D_tau
                                        removes and take their largest magnitude and the 1-norm of the
                                        removed part (the dropped matrices of eqs. 11 and 14, whose norms
                                        enter the error bound of eq. 23); turns the row skip off, so that
                                        every removed entry is computed */

#define FPS_FLAG_DENSE 0x40ull       /* compute a sparse product densely on the FP64 matrix cores when the
                                        modelled time of the dense product (n rounded up to 128) is below
                                        that of the sparse one (its multiply-adds at the rate of the row
                                        kernel its rows take) and three dense n x n operands fit the free
                                        device memory; the decision is taken per stage in the sizing
                                        evaluation.  The
                                        product is then summed in the matrix cores' order: results agree
                                        with the ordered sparse path to rounding (and entries within
                                        rounding of tau may be kept or dropped differently), not bit for
                                        bit.  Not with FPS_FLAG_DROP_STATS; not for batches */
#define FPS_FLAG_DENSE_EXACT 0x200ull /* dense paths that keep the sparse path's order of operations: a
                                        product whose work has gone dense runs as sparse rows times dense
                                        rows (one dense row of the right operand streamed per stored entry
                                        of the left) or as a dense product on the vector units with every
                                        entry's sum taken over k in order, whichever modelled time is
                                        lowest, when it is below the sparse one's and the dense operands
                                        fit the free device memory.  Each entry is the fma chain over the
                                        left row's entries in order with exact zeros added, so results are
                                        the sparse path's bit for bit.  FPS_FLAG_DENSE also considers
                                        these paths.  Not with FPS_FLAG_DROP_STATS; not for batches */
#define FPS_FLAG_NO_SMALL 0x80ull    /* keep every row on a 64-lane wavefront.  Without it, a stage of more
                                        than 8192 rows whose sizing evaluation found every row within 96
                                        structural entries and a 3072-column window runs later
                                        evaluations four rows per wavefront (16 lanes per row), with the
                                        same order of operations and so the same results bit for bit */

typedef struct ihipStream_t *fps_stream; /* same type as hipStream_t */

typedef struct {
    int64_t n;
    int64_t nnz;
    const int64_t *row_ptr; /* device, n+1 */
    const int32_t *col;     /* device, nnz */
    const double *val;      /* device, nnz */
} fps_csr_view;

typedef struct fps_plan_s *fps_plan;
typedef struct fps_matrix_s *fps_matrix;

/* filters (fps_filter_opts.filter) */
#define FPS_FILTER_FIXED 0    /* drop |x| < tau after every sparse product (Section 3.1.1) */
#define FPS_FILTER_ADAPTIVE 1 /* Algorithm 1 after every sparse product, thresholds of eq. 28 */

typedef struct {
    int32_t filter;         /* FPS_FILTER_FIXED or FPS_FILTER_ADAPTIVE */
    int32_t max_alg1_iters; /* adaptive: iteration limit of Algorithm 1 (0: 200) */
    double tau;             /* fixed: entry threshold (finite, >= 0) */
    double eps;             /* adaptive: filtering error budget epsilon of eq. 27 (> 0) */
    double e_r;             /* adaptive: Algorithm 1 tolerance e_r (>= 0) */
    const double *znorm;    /* adaptive: HOST array, znorm[t] >= ||Z^t||_1 for t = 0..max(s, s(b-1)),
                               b = ceil((m+1)/s); copied at plan time; NULL: the bounds of eq. 37
                               from fps_power_norm_bounds with K = 10 (synchronises at creation) */
    int32_t alg1_device_iters; /* adaptive: Algorithm 1 iterations launched per stage on the device
                                  without host synchronisation; 0: as many as the stage needed in
                                  the last host-driven run (the first evaluation runs host-driven,
                                  one synchronisation per iteration, and learns them); -1: always
                                  host-driven.  A stage that needs more than were launched makes
                                  the result query repeat the evaluation host-driven */
    int32_t reserved;
} fps_filter_opts;

/* stage kinds in fps_stats */
#define FPS_STAGE_POWER 0  /* P_{index} = D_tau(Z (x) P_{index-1})            (eq. 11) */
#define FPS_STAGE_BLOCK 1  /* Bhat_{index}, coefficient sum                     (eq. 13) */
#define FPS_STAGE_GSTEP 2  /* S_1 = Bhat_{b-2} + c_{(b-1)q} P_q, no filter       (eq. 14) */
#define FPS_STAGE_HORNER 3 /* S_{index} = D_tau(Bhat + P_q (x) S_{index-1})    (eq. 14) */

typedef struct {
    int32_t N, q, b, g, J, start; /* schedule (eq. 6; J = highest power formed) */
    int32_t n_spgemm;             /* sparse products per evaluation: q+b-2-g when b >= 2 (eq. 5) */
    int32_t n_stages;             /* stage records below */
    int64_t evals;                /* evaluations run on this plan */
    int64_t nnz_out;              /* stored entries of F after the last evaluation */
    int64_t products;             /* multiply-adds performed in the last evaluation */
    int64_t products_skipped;     /* multiply-adds avoided by the exact bound test */
    int64_t rows_skipped;         /* output rows proven empty by the bound test */
    int64_t rows_global;          /* rows handled by the device-memory kernel (more than 512 structural
                                     entries or a window wider than 6912 columns) */
    int64_t rows_wide;            /* rows handled by the wide shared-memory kernel (more than 320
                                     entries or a window wider than 6144 columns) */
    int64_t resizes;              /* evaluations that had to re-size a buffer */
    double bytes_algorithmic;     /* per evaluation, summed over stages: every operand entry read once and
                                     every kept entry written once at 12 bytes (8 value + 4 column), plus
                                     8 (n+1) bytes of row offsets per operand and output.  Only rows that
                                     are computed count: a product stage whose rows were all proven
                                     empty counts what its analysis reads (12 bytes per left-operand
                                     entry, the 16-byte summary of each referenced row and of each
                                     block term's row, the left operand's offsets), and one
                                     with some rows proven empty scales its right-operand and block
                                     bytes by the fraction of rows computed */
    double numeric_ms;            /* FPS_FLAG_TIMING: numeric-kernel time per evaluation
                                     (all stages), averaged over the sampled evaluations since the
                                     previous fps_get_stats call (up to 64; the latest sampled one if
                                     none) */
    int32_t numeric_launches;     /* FPS_FLAG_TIMING: stages timed per evaluation */
    int32_t kind[FPS_MAX_STAGES];
    int32_t index[FPS_MAX_STAGES];
    int64_t stage_products[FPS_MAX_STAGES];
    int64_t stage_nnz[FPS_MAX_STAGES]; /* kept entries of the stage output */
    double stage_ms[FPS_MAX_STAGES];   /* FPS_FLAG_TIMING: numeric-kernel time per stage, same average */
    /* adaptive filter, per stage (0 for stages without a sparse product) */
    double stage_eps_g[FPS_MAX_STAGES];     /* filtering-norm threshold of the stage (eq. 28) */
    double stage_threshold[FPS_MAX_STAGES]; /* final entry threshold of Algorithm 1 (|x| <= it dropped) */
    double stage_dropped[FPS_MAX_STAGES];   /* 1-norm of the dropped entries (integer column sums); with a
                                               fixed threshold and FPS_FLAG_DROP_STATS, the largest column
                                               sum of ceil(|x| 2^40 / tau) 2^-40 tau over the entries
                                               removed (an upper bound, within 2^-40 tau per entry) */
    int32_t stage_alg1_iters[FPS_MAX_STAGES];
    /* FPS_FLAG_DROP_STATS with a fixed threshold, per filtered product (0 otherwise) */
    int64_t stage_n_dropped[FPS_MAX_STAGES]; /* nonzero entries with |x| < tau removed */
    double stage_dropped_max[FPS_MAX_STAGES]; /* their largest magnitude */
    /* how Algorithm 1 ran on each stage in the last evaluation: 0 host-driven (or no Algorithm 1),
       1 on the device with the first iteration's sums taken in the product's write-out, 2 on the
       device with the drop of a one-iteration stage taken in the write-out, 3 on the device with
       the drop at the learned final threshold taken in the write-out, 4 on the device unfused */
    int32_t stage_alg1_mode[FPS_MAX_STAGES];
    int64_t stage_rows_skipped[FPS_MAX_STAGES]; /* output rows proven empty by the bound test */
    double stage_bytes[FPS_MAX_STAGES]; /* algorithmic bytes of the stage (see bytes_algorithmic) */
    int32_t stage_dense[FPS_MAX_STAGES];  /* the product ran on a dense path: 1 the matrix cores
                                             (FPS_FLAG_DENSE), 2 sparse rows times dense rows, 3 the
                                             ordered dense product on the vector units (2 and 3 exact:
                                             FPS_FLAG_DENSE_EXACT or FPS_FLAG_DENSE) */
    int64_t dense_ld;                     /* leading dimension of the dense operands (0 if none ran) */
    int32_t stage_small[FPS_MAX_STAGES];  /* 1: every row of the stage ran in the small-row tier, four rows
                                             per wavefront (see FPS_FLAG_NO_SMALL) */
    int64_t stage_max_ns[FPS_MAX_STAGES];    /* largest structural row (entries before the drop) seen by the
                                                stage's sizing evaluations */
    int64_t stage_max_words[FPS_MAX_STAGES]; /* widest row window, in 32-column words, seen by them */
} fps_stats;

/* ---------------------------------------------------------------------- */
/* Version and errors                                                       */
/* ---------------------------------------------------------------------- */

int32_t fps_abi_version(void);
const char *fps_status_string(fps_status s);
/* Thread-local text of the last error on this thread ("" if none).  The
 * pointer stays valid until the next fps_* call on the same thread. */
const char *fps_last_error(void);

/* Schedule of eq. 6 with q = s given (host only, no device work).  Any
 * output pointer may be NULL.  INVALID_ARG if m < 0 or s < 1. */
fps_status fps_schedule(int32_t m, int32_t s, int32_t *N, int32_t *q, int32_t *b, int32_t *g, int32_t *J,
                        int32_t *start, int32_t *n_spgemm);

/* ---------------------------------------------------------------------- */
/* Plan / evaluate (Algorithm 2 with a fixed tau)                           */
/* ---------------------------------------------------------------------- */

/*
 * Create a plan for F(Z) with coefficients coeffs[0..m] (HOST array, copied),
 * PS block size s (1 <= s <= FPS_MAX_S) and filter threshold tau (finite,
 * >= 0; tau = 0 drops exact zeros only, i.e. the unfiltered PS scheme).
 * Z is borrowed: its device arrays must stay valid and unchanged while any
 * fps_eval of this plan is in flight.  Unless FPS_FLAG_NO_VALIDATE is set,
 * Z is checked on the device (synchronising `stream`); failure gives
 * FPS_ERR_BAD_CSR.  The plan owns all device workspace.
 */
fps_status fps_plan_create(fps_plan *out, const fps_csr_view *Z, const double *coeffs, int32_t m, int32_t s,
                           double tau, uint64_t flags, fps_stream stream);

/*
 * Same as fps_plan_create with the filter chosen by `opts`.  With
 * FPS_FILTER_ADAPTIVE every sparse product (powers, eq. 11; Horner steps,
 * eq. 14) is formed without filtering and then filtered by Algorithm 1 with
 * eps_g = zeta_k or sigma_j of eq. 28 (computed from eqs. 21-26 with the given
 * norm bounds), so that the filtering error is at most eps (1 + e_r) to first
 * order (eq. 27).  Algorithm 1 measures the candidate norm as the largest
 * column sum of ceil(|x| 2^40 / eps_g) taken exactly in integers (an upper
 * bound of the 1-norm, independent of summation order).  The iterations of
 * Algorithm 1 run on the device (opts->alg1_device_iters), so an evaluation
 * only enqueues work once the plan has learned its sizes.
 */
fps_status fps_plan_create_ex(fps_plan *out, const fps_csr_view *Z, const double *coeffs, int32_t m, int32_t s,
                              const fps_filter_opts *opts, uint64_t flags, fps_stream stream);

/* ---- Series mode (Section 3.2; Algorithm 2 steps 1-3; eqs. 33-37) ------- */

/*
 * Estimate of ||Z^p||_1 by the block 1-norm estimator of Higham and Tisseur
 * (the estimator behind normest1, which the paper uses for eq. 37) with one
 * column and at most 5 iterations, A = Z^p applied as p products with Z (A x)
 * or Z^T (A^T s): start vector ones/n, sign(0) = +1, among equal largest
 * |(A^T s)_i| the smallest i.  Every product accumulates in ascending index
 * order with fused multiply-adds from +0, and ||y||_1 adds |y_i| in ascending
 * index order from +0, so the result is reproducible bit for bit.
 * *est <= ||Z^p||_1 and *est =
 * ||Z^p v||_1 for v = e_{*ind} (*ind = -1: the start vector won).  Z: device
 * CSR view, checked unless FPS_FLAG_NO_VALIDATE; est, ind, iters: HOST
 * pointers (ind, iters may be NULL).  p >= 0.  Synchronises `stream`.
 */
fps_status fps_normest1(const fps_csr_view *Z, int32_t p, double *est, int64_t *ind, int32_t *iters, uint64_t flags,
                        fps_stream stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * estimate as fps_normest1, bit for bit, with every piece of device workspace
 * (the transpose of Z, the iteration vectors, the validation flag) in a
 * static buffer of the library instead of allocations.  The buffer holds
 * about 16.5 MiB per GPU (sized for FPS_NOALLOC_MAX_N rows and
 * FPS_NOALLOC_MAX_NNZ entries), is set up on the first call on each device
 * and kept until the process ends; no call allocates or frees device memory.
 * FPS_ERR_CAPACITY if n > FPS_NOALLOC_MAX_N or nnz > FPS_NOALLOC_MAX_NNZ.
 * Every call on one GPU uses the same buffer: calls that overlap on one GPU
 * (from several host threads, or on several streams without ordering between
 * them) race and give undefined results.  Arguments, synchronisation and
 * errors as for fps_normest1.
 */
#define FPS_NOALLOC_MAX_N 65536
#define FPS_NOALLOC_MAX_NNZ 524288
fps_status fps_normest1_noalloc(const fps_csr_view *Z, int32_t p, double *est, int64_t *ind, int32_t *iters,
                                uint64_t flags, fps_stream stream);

/*
 * Norm bounds of eq. 37 into the HOST array z[0..tmax]: z[0] = 1,
 * z[i] = fps_normest1(Z, i) for 1 <= i <= K, z[i] = alpha^i for i > K with
 * alpha = max over k = K/2..K of z[k]^(1/k) (Lemma 1).  K even and >= 2 (the
 * paper takes K = 10).  Synchronises `stream`.
 */
fps_status fps_power_norm_bounds(const fps_csr_view *Z, int32_t K, int32_t tmax, double *z, uint64_t flags,
                                 fps_stream stream);

typedef struct {
    double eps_tol;          /* error tolerance of Algorithm 2 (> 0) */
    double e_r;              /* Algorithm 1 tolerance (>= 0) */
    int32_t K;               /* eq. 37 estimate depth, even (0: 10) */
    int32_t max_alg1_iters;  /* Algorithm 1 iteration limit (0: 200) */
    int32_t alg1_device_iters; /* as in fps_filter_opts */
    int32_t reserved;
} fps_series_opts;

/*
 * A plan for the power series f(Z) = sum_i a_i Z^i given by its first L
 * coefficients a[0..L-1] (HOST; terms beyond are taken as zero), evaluated so
 * that ||f(Z) - F||_1 <= eps_tol (Algorithm 2): z[0..L-1] by eq. 37; N = the
 * smallest m >= 1 with T_m = sum_{i >= m} |a_i| z_i <= eps_tol / 2 (eq. 34;
 * T accumulated from the end, T_L = 0); q = floor(sqrt(N - 1)), at least 1
 * (Algorithm 2 step 3); then the plan of fps_plan_create_ex for the degree
 * N - 1 polynomial with block size q, FPS_FILTER_ADAPTIVE and the budget
 * eps_tol - T_N, which makes its eq. 28 thresholds those of eq. 36.
 * FPS_ERR_INVALID_ARG if N would reach L (more coefficients are needed),
 * FPS_ERR_CAPACITY if q > FPS_MAX_S.  The estimation runs here and
 * synchronises `stream`; evaluation as for any plan.
 */
fps_status fps_plan_create_series(fps_plan *out, const fps_csr_view *Z, const double *a, int32_t L,
                                  const fps_series_opts *opts, uint64_t flags, fps_stream stream);

/* The quantities of a series plan: N (eq. 34), q (Algorithm 2 step 3), the
 * tail T_N (eq. 33), the filtering budget eps_tol - T_N and, into the optional
 * HOST array z[0..L-1], the eq. 37 bounds.  FPS_ERR_INVALID_ARG for a plan not
 * made by fps_plan_create_series.  Host only. */
fps_status fps_plan_series_info(fps_plan p, int32_t *N, int32_t *q, double *tail, double *budget, double *z);

/*
 * Evaluate F(Z) on `stream`.  Once the plan has learned its buffer sizes
 * (after its first evaluation, or always with FPS_FLAG_SYNC_SIZES) this only
 * enqueues work; otherwise it synchronises `stream` once per stage to size
 * the outputs.  If Z's values changed so that a learned size no longer fits,
 * the kernels flag it and fps_result_nnz re-runs the evaluation with sizing.
 */
fps_status fps_eval(fps_plan p, fps_stream stream);

/* Number of stored entries of F (synchronises the plan's last stream).
 * NOT_READY before the first fps_eval. */
fps_status fps_result_nnz(fps_plan p, int64_t *nnz);

/* Copy F as canonical CSR into caller-owned DEVICE buffers: row_ptr int64[n+1],
 * col int32[nnz], val double[nnz] with nnz from fps_result_nnz.  Enqueued on
 * `stream` after the evaluation. */
fps_status fps_result_copy(fps_plan p, int64_t *row_ptr, int32_t *col, double *val, fps_stream stream);

/* Statistics of the last evaluation (synchronises). */
fps_status fps_get_stats(fps_plan p, fps_stats *st);

/* Release the plan and its workspace (synchronises its stream first). */
void fps_plan_destroy(fps_plan p);

/* ---------------------------------------------------------------------- */
/* Single stages (the building blocks of fps_eval, for tests and tools)     */
/* ---------------------------------------------------------------------- */

/*
 * C = D_tau(E + A (x) B): one filtered sparse product with an optional extra
 * matrix E added to the product before the drop test (eq. 11 with E = NULL,
 * one step of eq. 14 with E = Bhat).  A, B, E are n x n canonical CSR (E may
 * be NULL).  The result is a library-owned canonical CSR matrix.
 * Synchronises `stream` (to size the output).
 */
fps_status fps_spgemm(fps_matrix *out, const fps_csr_view *A, const fps_csr_view *B, const fps_csr_view *E,
                      double tau, fps_stream stream);

/*
 * C = sum_t coefs[t] * M_t accumulated in the order t = 0..nterms-1 (eq. 13);
 * exact zeros are dropped, nothing else.  coefs is a HOST array; terms[t] is a
 * canonical n x n CSR view, or the identity when terms[t].row_ptr == NULL.
 * 1 <= nterms <= FPS_MAX_S + 1.  Synchronises `stream`.
 */
fps_status fps_axpy(fps_matrix *out, int64_t n, int32_t nterms, const double *coefs, const fps_csr_view *terms,
                    fps_stream stream);

fps_status fps_matrix_nnz(fps_matrix m, int64_t *nnz);
/* Copy a library matrix into caller-owned DEVICE buffers (see fps_result_copy). */
fps_status fps_matrix_copy(fps_matrix m, int64_t *row_ptr, int32_t *col, double *val, fps_stream stream);
void fps_matrix_destroy(fps_matrix m);

/* ---------------------------------------------------------------------- */
/* Batch: many evaluations in one launch sequence                          */
/* ---------------------------------------------------------------------- */

typedef struct fps_batch_s *fps_batch;

typedef struct {
    fps_csr_view Z;         /* device CSR, borrowed (as for fps_plan_create) */
    const double *coeffs;   /* HOST, m+1 entries, copied */
    int32_t m;              /* degree */
    int32_t s;              /* PS block size; 0: chosen by fps_autotune_s in [s_lo, s_hi] */
    double tau;             /* fixed threshold of this instance (finite, >= 0) */
} fps_batch_item;

#define FPS_BATCH_NO_GRAPH 0x100ull /* batch flag: evaluate with ordinary launches, no graph replay */

/*
 * A batch of `count` independent filtered PS evaluations (each as
 * fps_plan_create would do it with its own Z, coefficients, m, s and tau).
 * Instances with the same m, s and coefficients form a group whose matrices
 * are joined into one block-diagonal CSR (rows of instance i after those of
 * the instances before it, columns shifted alike) with a per-row threshold;
 * every stage of the scheme is then one launch over all the group's rows,
 * and since an output row only reads rows of its own block, each instance's
 * result equals its own plan's bit for bit.
 * Autotuner: items with s == 0 get the block size in [s_lo, s_hi] (s_lo =
 * s_hi = 0: floor(sqrt(m)) - 1 .. floor(sqrt(m)) + 1, at least 1) whose
 * evaluation takes the fewest multiply-adds, measured by one sizing
 * evaluation per candidate of the instances with the same series joined
 * (ties: the smaller s).  The paper's optimal q (eqs. 5-6) minimises the
 * number of matrix products; for sparse operands the powers grow denser and
 * the products differ in cost, so the count of scalar multiply-adds is what
 * is minimised.  It is an exact integer of the instance alone, so the choice
 * is deterministic and does not depend on the other items.  Each Z is
 * validated on the device unless
 * FPS_FLAG_NO_VALIDATE; FPS_FLAG_NO_SKIP and FPS_FLAG_FORCE_GLOBAL apply to
 * every group, FPS_FLAG_DROP_STATS is not supported.  The joined copies are
 * made here: the Z arrays need not stay valid afterwards.  The total number
 * of rows of a group is at most FPS_MAX_N.  Synchronises `stream`.
 */
fps_status fps_batch_create(fps_batch *out, const fps_batch_item *items, int32_t count, int32_t s_lo, int32_t s_hi,
                            uint64_t flags, fps_stream stream);

/*
 * Evaluate every instance on `stream`.  The first call sizes the groups'
 * buffers (host reads, as a plan's first evaluation) and the second runs with
 * ordinary launches (it may still grow a buffer); from the third on, calls
 * replay one captured HIP graph in which the groups run as parallel branches
 * (unless FPS_BATCH_NO_GRAPH), with no host synchronisation.  A capacity flag raised
 * in a replay is handled by the next result query (the evaluation is
 * repeated with sizing and the graph captured again).
 */
fps_status fps_batch_eval(fps_batch b, fps_stream stream);

/* Stored entries of instance i's result (synchronises). */
fps_status fps_batch_result_nnz(fps_batch b, int32_t i, int64_t *nnz);

/* Copy instance i's result as canonical CSR into caller-owned DEVICE buffers
 * (row_ptr int64[n_i + 1], col int32[nnz], val double[nnz]); enqueued on
 * `stream`. */
fps_status fps_batch_result_copy(fps_batch b, int32_t i, int64_t *row_ptr, int32_t *col, double *val,
                                 fps_stream stream);

typedef struct {
    int32_t count;            /* instances */
    int32_t groups;           /* groups (distinct m, s, coefficients) */
    int32_t graph;            /* 1 if evaluations replay a captured graph */
    int32_t reserved;
    int64_t evals;            /* evaluations run */
    int64_t graph_launches;   /* of which graph replays */
    int64_t resizes;          /* evaluations repeated with sizing */
    int64_t rows;             /* rows over all instances */
    int64_t nnz_out;          /* stored entries over all results of the last evaluation */
    int64_t products;         /* multiply-adds of the last evaluation over all groups */
    double bytes_algorithmic; /* over all groups (see fps_stats) */
} fps_batch_stats;

/* Statistics of the batch (synchronises). */
fps_status fps_batch_get_stats(fps_batch b, fps_batch_stats *st);

/* Block size and group of instance i, and (if it was tuned) into the HOST
 * array products[0 .. s_hi - s_lo] its measured multiply-adds for each
 * candidate s (host only). */
fps_status fps_batch_item_info(fps_batch b, int32_t i, int32_t *s, int32_t *group, int64_t *products);

/* Release the batch (synchronises its last stream). */
void fps_batch_destroy(fps_batch b);

/* ---------------------------------------------------------------------- */
/* Server: continuous admission of evaluations by device-memory footprint  */
/* ---------------------------------------------------------------------- */

typedef struct fps_server_s *fps_server;

typedef struct {
    int32_t slots;        /* worker slots (1..64), each a host thread with its own stream: up to `slots`
                             requests run at once and their kernels overlap on the device */
    int32_t max_queue;    /* waiting requests accepted before fps_server_submit refuses (0: 4096) */
    int64_t hbm_budget;   /* device bytes that the running requests may reserve and the finished,
                             unreleased results may hold, in total (> 0) */
    uint64_t flags;       /* plan flags applied to every request (FPS_FLAG_NO_VALIDATE, FPS_FLAG_NO_SKIP,
                             FPS_FLAG_DENSE, FPS_FLAG_DENSE_EXACT) */
    int32_t fake_backend; /* 1: nothing is computed and no device call is made: a worker holds each request
                             for n microseconds and charges 100 n bytes against its reservation (tests of
                             the scheduler without a GPU) */
    int32_t no_grow;      /* 1: a request that needs more than its reservation always runs again with a
                             larger one; 0: it first grows the reservation in place (see below) */
} fps_server_opts;

/* request states */
#define FPS_REQ_QUEUED 0
#define FPS_REQ_RUNNING 1
#define FPS_REQ_DONE 2
#define FPS_REQ_FAILED 3

/*
 * A server of fixed-threshold filtered PS evaluations (each as
 * fps_plan_create + fps_eval would run it).  Requests wait in one FIFO queue;
 * the head is admitted when a slot is free and its reservation fits the
 * budget beside the reservations of the running requests and the bytes of
 * the finished results not yet released.  A request's plan may hold at most
 * its reservation (an estimate from n, nnz, m and s, or the caller's hint).
 * If it needs more, the reservation grows in place, to a quarter more than
 * needed, when the budget has room for that beside everything else reserved
 * or held (unless opts->no_grow), and the run goes on; otherwise the request
 * goes back to the head of the queue with four times the reservation (up to
 * the whole budget) and runs again when that fits.
 * A finished request keeps only its result (canonical CSR) on the device
 * until fps_server_release.  Results do not depend on what else runs: each
 * request is its own plan, evaluated exactly as alone.
 */
fps_status fps_server_create(fps_server *out, const fps_server_opts *opts);

/*
 * Queue an evaluation: Z (device CSR, borrowed until the request is done or
 * failed), coefficients c[0..m] (HOST, copied), block size s (0: floor(sqrt(m)),
 * the q of eq. 6, at least 1), threshold tau; reserve_hint > 0 sets the first
 * reservation in bytes.  *ticket identifies the request.  FPS_ERR_CAPACITY
 * when max_queue requests are waiting (the caller retries later).
 */
fps_status fps_server_submit(fps_server sv, const fps_csr_view *Z, const double *coeffs, int32_t m, int32_t s,
                             double tau, int64_t reserve_hint, int64_t *ticket);

/* Wait until the request is done or failed, or timeout_ms passes (< 0: no
 * limit); *state gets its state.  The request's own status is in
 * fps_server_request_info. */
fps_status fps_server_wait(fps_server sv, int64_t ticket, int64_t timeout_ms, int32_t *state);

/* The result of a done request: entries, and a copy into caller-owned DEVICE
 * buffers (row_ptr int64[n + 1], col int32[nnz], val double[nnz]) enqueued on
 * `stream`.  FPS_ERR_NOT_READY unless done. */
fps_status fps_server_result_nnz(fps_server sv, int64_t ticket, int64_t *nnz);
fps_status fps_server_result_copy(fps_server sv, int64_t ticket, int64_t *row_ptr, int32_t *col, double *val,
                                  fps_stream stream);

/* Forget a done or failed request and free its result (after the copies
 * out of it enqueued by fps_server_result_copy have finished). */
fps_status fps_server_release(fps_server sv, int64_t ticket);

typedef struct {
    int32_t state;       /* FPS_REQ_* */
    int32_t status;      /* fps_status of a finished request */
    int32_t attempts;    /* runs (more than one after a reservation was too small) */
    int32_t s;           /* block size used */
    int64_t n;
    int64_t reserve;     /* current reservation, bytes */
    int64_t held;        /* bytes of the kept result (done requests) */
    int64_t peak;        /* largest device bytes its plan held */
    int64_t t_submit_ns; /* steady-clock times: submission, start of the last run, result ready */
    int64_t t_start_ns;
    int64_t t_done_ns;
} fps_server_request;

fps_status fps_server_request_info(fps_server sv, int64_t ticket, fps_server_request *out);

typedef struct {
    int64_t submitted, completed, failed, retries, refused;
    int32_t running, queued, slots, peak_running;
    int64_t reserved;      /* bytes reserved now (running) or held (finished, unreleased) */
    int64_t peak_reserved; /* its largest value so far (never above the budget) */
    int64_t budget;
    int64_t grows;         /* reservations grown in place */
} fps_server_stats;

fps_status fps_server_get_stats(fps_server sv, fps_server_stats *out);

/* Stop the server: running requests finish, waiting ones fail; then free
 * everything (results included). */
void fps_server_destroy(fps_server sv);

#ifdef __cplusplus
}
#endif

#endif /* FPS_H */
