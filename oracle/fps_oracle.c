/*
 * CPU oracle for the filtered Paterson-Stockmeyer (PS) evaluation of a
 * matrix power series  F(Z) = sum_{k=0..m} c_k Z^k  on a sparse Z.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it exists so that tests and the CPU-baseline timing can
 * check the HIP implementation against a plain, slow, obviously correct
 * version written from the paper.  It shares no code with the HIP path.
 *
 * Paper: "A filtering technique for the matrix power series being
 * near-sparse" (arXiv 2208.05683).
 *
 * What is computed (paper Section 2.1 eqs. 2-6, Section 3.1.2 eqs. 11, 13,
 * 14, Algorithm 2 with a fixed entry threshold tau in place of the adaptive
 * filter of Algorithm 1; the plain fixed-threshold filter that Section
 * 3.1.1 describes before it):
 *
 *   N = m+1, q = s, b = ceil(N/q), g = [N - q(b-1) == 1]          (eq. 6)
 *   P_1 = Z,  P_{j+1} = D_tau(Z (x) P_j)                            (eq. 11)
 *   Bhat_i = sum_{j<q} c_{iq+j} P_j,  P_0 = I, not filtered          (eq. 13)
 *   S_0 = Bhat_{b-1};  if g: S_1 = Bhat_{b-2} + c_{(b-1)q} P_q,
 *                           no product and no filter                (eq. 14)
 *   S_i = D_tau(Bhat_{b-1-i} + P_q (x) S_{i-1})                     (eq. 14)
 *   F   = S_{b-1}
 *
 * Readings of points the paper leaves open (fixed here, shared by every
 * implementation that claims parity with this file):
 *   - D_tau drops an entry x iff x == 0 or |x| < tau (|x| == tau is kept);
 *     exact zeros are dropped everywhere, also where nothing is filtered.
 *   - (x) is Gustavson's row-wise product: for output row r, for the stored
 *     k of row r of the left operand in ascending order, acc += a_rk * B_k,:
 *     with one fused multiply-add per term, acc starting at +0.
 *   - Bhat_i and the g-shortcut sum accumulate the terms c_j P_j in
 *     ascending j with fused multiply-adds from +0; terms with c_j == 0
 *     are skipped.  The g-shortcut sum is Bhat_{b-2} extended by the term
 *     j = q, i.e. sum_{j=0..q} c_{(b-2)q+j} P_j in one ascending pass.
 *   - In a Horner step the block enters with one addition: x = bhat + prod.
 *   - The left factor is Z for the powers (eq. 11) and P_q for the Horner
 *     steps (eq. 14), as the paper writes them.
 *   - Powers are formed up to J = q when b >= 2, else up to J = m.
 *
 * Rows are independent; OpenMP splits rows across threads for timing only.
 * Each row is computed by one thread in the order above, so results do not
 * depend on the thread count.  Only the dropped-norm statistic (a sum over
 * rows per column) may differ in its last bits between thread counts.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int64_t n;
    int64_t nnz;
    int64_t *row_ptr; /* n+1 */
    int32_t *col;     /* nnz, sorted and unique per row */
    double *val;      /* nnz */
} orc_csr;

typedef struct {
    int32_t kind;   /* 0 power P_{index}, 1 block Bhat_{index}, 2 g-shortcut S_1, 3 Horner S_{index} */
    int32_t index;
    int64_t products;    /* scalar multiply-adds of the product part */
    int64_t nnz_struct;  /* distinct structural entries before dropping */
    int64_t nnz_kept;
    int64_t n_dropped;   /* nonzero entries removed by the tau test */
    int64_t n_zero;      /* entries removed because they were exactly zero */
    double dropped_1norm; /* max over columns of the sum of |dropped| */
    double dropped_max;   /* largest |dropped| (0 if none) */
    double kept_min;      /* smallest |kept| (inf if none) */
} orc_stage_stats;

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_ENOMEM = 3 };

/* ------------------------------------------------------------------ */
/* small helpers                                                        */
/* ------------------------------------------------------------------ */

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

void orc_csr_free(orc_csr *m)
{
    if (!m) return;
    free(m->row_ptr);
    free(m->col);
    free(m->val);
    m->row_ptr = NULL;
    m->col = NULL;
    m->val = NULL;
    m->nnz = 0;
}

static int nthreads_or_default(int nt)
{
#ifdef _OPENMP
    return nt > 0 ? nt : omp_get_max_threads();
#else
    (void)nt;
    return 1;
#endif
}

/* per-thread growable output of kept entries */
typedef struct {
    int32_t *col;
    double *val;
    int64_t len, cap;
} rowbuf;

static int rowbuf_push(rowbuf *b, int32_t c, double v)
{
    if (b->len == b->cap) {
        int64_t nc = b->cap ? 2 * b->cap : 1024;
        int32_t *c2 = realloc(b->col, (size_t)nc * sizeof(int32_t));
        if (!c2) return -1;
        b->col = c2;
        double *v2 = realloc(b->val, (size_t)nc * sizeof(double));
        if (!v2) return -1;
        b->val = v2;
        b->cap = nc;
    }
    b->col[b->len] = c;
    b->val[b->len] = v;
    b->len++;
    return 0;
}

/*
 * One "term source" per output row: the generic row computation below is
 *     x[c] = extra[c] + sum_t  a_t * R_t[c]
 * accumulated term by term in the given order with fma from +0, then the
 * extra row (if any) enters with one addition, then the drop test.
 * For a product A (x) B the terms of row r are (A_rk, B_k,:) over k in A_r;
 * for a coefficient sum they are (c_j, P_j[r,:]).
 */
typedef struct {
    /* mode 0: product; mode 1: coefficient sum */
    int mode;
    const orc_csr *A, *B;      /* product operands */
    int nterms;
    const double *coef;        /* coefficient-sum weights */
    const orc_csr *const *mat; /* coefficient-sum matrices; NULL = identity */
    const orc_csr *extra;      /* row added after the products (may be NULL) */
    double tau;                /* drop |x| < tau; 0 drops exact zeros only */
    int64_t n;
} orc_job;

typedef struct {
    double *acc;
    int64_t *mark; /* mark[c] == r+1 if column c touched in row r */
    int32_t *list;
    double *drop_colsum;
    rowbuf out;
    int64_t products, nnz_struct, n_dropped, n_zero;
    double dropped_max, kept_min;
    int err;
} orc_ws;

static void compute_row(const orc_job *jb, orc_ws *w, int64_t r, int64_t *row_off, int64_t *row_len)
{
    int64_t nl = 0;
    const int64_t tag = r + 1;
#define TOUCH(c)                                  \
    do {                                          \
        if (w->mark[(c)] != tag) {                \
            w->mark[(c)] = tag;                   \
            w->acc[(c)] = 0.0;                    \
            w->list[nl++] = (int32_t)(c);         \
        }                                         \
    } while (0)

    if (jb->mode == 0) {
        const orc_csr *A = jb->A, *B = jb->B;
        for (int64_t p = A->row_ptr[r]; p < A->row_ptr[r + 1]; ++p) {
            const int64_t k = A->col[p];
            const double a = A->val[p];
            for (int64_t t = B->row_ptr[k]; t < B->row_ptr[k + 1]; ++t) {
                const int32_t c = B->col[t];
                TOUCH(c);
                w->acc[c] = fma(a, B->val[t], w->acc[c]);
                w->products++;
            }
        }
    } else {
        for (int t = 0; t < jb->nterms; ++t) {
            const double a = jb->coef[t];
            const orc_csr *M = jb->mat[t];
            if (M == NULL) { /* identity: row r has the single entry (r, 1) */
                TOUCH(r);
                w->acc[r] = fma(a, 1.0, w->acc[r]);
                w->products++;
            } else {
                for (int64_t p = M->row_ptr[r]; p < M->row_ptr[r + 1]; ++p) {
                    const int32_t c = M->col[p];
                    TOUCH(c);
                    w->acc[c] = fma(a, M->val[p], w->acc[c]);
                    w->products++;
                }
            }
        }
    }
    if (jb->extra) {
        const orc_csr *E = jb->extra;
        for (int64_t p = E->row_ptr[r]; p < E->row_ptr[r + 1]; ++p) {
            const int32_t c = E->col[p];
            TOUCH(c);
            w->acc[c] = E->val[p] + w->acc[c];
        }
    }
#undef TOUCH
    qsort(w->list, (size_t)nl, sizeof(int32_t), cmp_i32);
    w->nnz_struct += nl;
    *row_off = w->out.len;
    for (int64_t i = 0; i < nl; ++i) {
        const int32_t c = w->list[i];
        const double x = w->acc[c];
        if (x == 0.0) {
            w->n_zero++;
            continue;
        }
        if (fabs(x) < jb->tau) {
            w->n_dropped++;
            w->drop_colsum[c] += fabs(x);
            if (fabs(x) > w->dropped_max) w->dropped_max = fabs(x);
            continue;
        }
        if (fabs(x) < w->kept_min) w->kept_min = fabs(x);
        if (rowbuf_push(&w->out, c, x)) w->err = 1;
    }
    *row_len = w->out.len - *row_off;
}

static int run_job(const orc_job *jb, orc_csr *C, orc_stage_stats *st, int nthreads)
{
    const int64_t n = jb->n;
    const int nt = nthreads_or_default(nthreads);
    orc_ws *ws = calloc((size_t)nt, sizeof(orc_ws));
    int64_t *off = malloc((size_t)(n + 1) * sizeof(int64_t));
    int64_t *len = malloc((size_t)(n + 1) * sizeof(int64_t));
    int32_t *owner = malloc((size_t)(n + 1) * sizeof(int32_t));
    if (!ws || !off || !len || !owner) {
        free(ws); free(off); free(len); free(owner);
        return ORC_ENOMEM;
    }
    int err = 0;
    for (int t = 0; t < nt; ++t) {
        ws[t].acc = malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
        ws[t].mark = calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
        ws[t].list = malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
        ws[t].drop_colsum = calloc((size_t)(n > 0 ? n : 1), sizeof(double));
        ws[t].kept_min = INFINITY;
        if (!ws[t].acc || !ws[t].mark || !ws[t].list || !ws[t].drop_colsum) err = 1;
    }
    if (!err) {
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
        {
#ifdef _OPENMP
            const int t = omp_get_thread_num();
#else
            const int t = 0;
#endif
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
            for (int64_t r = 0; r < n; ++r) {
                compute_row(jb, &ws[t], r, &off[r], &len[r]);
                owner[r] = t;
            }
        }
    }
    for (int t = 0; t < nt; ++t) err |= ws[t].err;
    if (!err) {
        C->n = n;
        C->row_ptr = malloc((size_t)(n + 1) * sizeof(int64_t));
        if (!C->row_ptr) err = 1;
    }
    if (!err) {
        C->row_ptr[0] = 0;
        for (int64_t r = 0; r < n; ++r) C->row_ptr[r + 1] = C->row_ptr[r] + len[r];
        C->nnz = C->row_ptr[n];
        C->col = malloc((size_t)(C->nnz > 0 ? C->nnz : 1) * sizeof(int32_t));
        C->val = malloc((size_t)(C->nnz > 0 ? C->nnz : 1) * sizeof(double));
        if (!C->col || !C->val) err = 1;
    }
    if (!err) {
        for (int64_t r = 0; r < n; ++r) {
            const rowbuf *b = &ws[owner[r]].out;
            memcpy(C->col + C->row_ptr[r], b->col + off[r], (size_t)len[r] * sizeof(int32_t));
            memcpy(C->val + C->row_ptr[r], b->val + off[r], (size_t)len[r] * sizeof(double));
        }
        if (st) {
            memset(st, 0, sizeof(*st));
            st->kept_min = INFINITY;
            double *colsum = calloc((size_t)(n > 0 ? n : 1), sizeof(double));
            if (!colsum) err = 1;
            for (int t = 0; t < nt && !err; ++t) {
                st->products += ws[t].products;
                st->nnz_struct += ws[t].nnz_struct;
                st->n_dropped += ws[t].n_dropped;
                st->n_zero += ws[t].n_zero;
                if (ws[t].dropped_max > st->dropped_max) st->dropped_max = ws[t].dropped_max;
                if (ws[t].kept_min < st->kept_min) st->kept_min = ws[t].kept_min;
                for (int64_t c = 0; c < n; ++c) colsum[c] += ws[t].drop_colsum[c];
            }
            if (!err) {
                double mx = 0.0;
                for (int64_t c = 0; c < n; ++c)
                    if (colsum[c] > mx) mx = colsum[c];
                st->dropped_1norm = mx;
                st->nnz_kept = C->nnz;
            }
            free(colsum);
        }
    }
    for (int t = 0; t < nt; ++t) {
        free(ws[t].acc); free(ws[t].mark); free(ws[t].list); free(ws[t].drop_colsum);
        free(ws[t].out.col); free(ws[t].out.val);
    }
    free(ws); free(off); free(len); free(owner);
    if (err) {
        orc_csr_free(C);
        return ORC_ENOMEM;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* single stages                                                        */
/* ------------------------------------------------------------------ */

/*
 * C = D_tau(E + A (x) B): one filtered product (eq. 11 with E absent,
 * eq. 14 with E = Bhat).  tau = 0 drops exact zeros only.
 */
int orc_spgemm(const orc_csr *A, const orc_csr *B, const orc_csr *E, double tau,
               orc_csr *C, orc_stage_stats *st, int nthreads)
{
    if (!A || !B || !C || A->n != B->n || (E && E->n != A->n) || !(tau >= 0.0)) return ORC_EINVAL;
    orc_job jb = {0};
    jb.mode = 0;
    jb.A = A;
    jb.B = B;
    jb.extra = E;
    jb.tau = tau;
    jb.n = A->n;
    return run_job(&jb, C, st, nthreads);
}

/*
 * C = sum_t coef[t] * M_t in the given order (M_t == NULL means I), exact
 * zeros dropped, nothing else (eq. 13: the blocks are not filtered).
 */
int orc_axpy(int64_t n, int nterms, const double *coef, const orc_csr *const *mats,
             orc_csr *C, orc_stage_stats *st, int nthreads)
{
    if (!C || n < 0 || nterms < 0) return ORC_EINVAL;
    for (int t = 0; t < nterms; ++t)
        if (mats[t] && mats[t]->n != n) return ORC_EINVAL;
    orc_job jb = {0};
    jb.mode = 1;
    jb.nterms = nterms;
    jb.coef = coef;
    jb.mat = mats;
    jb.tau = 0.0;
    jb.n = n;
    return run_job(&jb, C, st, nthreads);
}

/* ------------------------------------------------------------------ */
/* schedule (eqs. 5-6 with q = s given)                                 */
/* ------------------------------------------------------------------ */

int orc_schedule(int m, int s, int *N, int *q, int *b, int *g, int *J, int *start, int *n_spgemm)
{
    if (m < 0 || s < 1) return ORC_EINVAL;
    const int NN = m + 1, qq = s, bb = (NN + qq - 1) / qq;
    const int gg = (NN - qq * (bb - 1) == 1) ? 1 : 0;
    const int JJ = (bb >= 2) ? qq : m;
    *N = NN; *q = qq; *b = bb; *g = gg; *J = JJ;
    *start = (bb >= 2) ? 1 + gg : 0;
    *n_spgemm = (JJ >= 1 ? JJ - 1 : 0) + (bb >= 2 ? bb - 1 - gg : 0);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* the filtered PS evaluation (Algorithm 2 with a fixed tau)             */
/* ------------------------------------------------------------------ */

static void record(orc_stage_stats *stats, int max_stats, int *ns, const orc_stage_stats *st,
                   int kind, int index)
{
    if (*ns < max_stats) {
        stats[*ns] = *st;
        stats[*ns].kind = kind;
        stats[*ns].index = index;
    }
    (*ns)++;
}

/* block i of eq. 13 extended to the coefficient indices [lo, hi] of the
 * series: sum over j with lo <= i*q+j <= hi of c_{iq+j} P_j, ascending j. */
static int coefficient_block(const orc_csr *const *P, const double *c, int m, int q, int i, int jmax,
                             int64_t n, orc_csr *out, orc_stage_stats *st, int nthreads)
{
    double coef[256];
    const orc_csr *mats[256];
    int nt = 0;
    for (int j = 0; j <= jmax; ++j) {
        const int k = i * q + j;
        if (k > m) break;
        if (c[k] == 0.0) continue;
        if (nt >= 256) return ORC_EINVAL;
        coef[nt] = c[k];
        mats[nt] = (j == 0) ? NULL : P[j];
        nt++;
    }
    return orc_axpy(n, nt, coef, mats, out, st, nthreads);
}

int orc_filtered_ps(const orc_csr *Z, const double *c, int m, int s, double tau, orc_csr *F,
                    orc_stage_stats *stats, int max_stats, int *n_stats, int nthreads)
{
    int N, q, b, g, J, start, nsp;
    if (!Z || !c || !F || !(tau >= 0.0) || orc_schedule(m, s, &N, &q, &b, &g, &J, &start, &nsp))
        return ORC_EINVAL;
    if (q > 255) return ORC_EINVAL;
    const int64_t n = Z->n;
    int ns = 0, rc = ORC_OK;
    orc_stage_stats st;
    orc_csr *P = calloc((size_t)(J + 2), sizeof(orc_csr));
    const orc_csr **Pp = calloc((size_t)(J + 2), sizeof(orc_csr *));
    if (!P || !Pp) { free(P); free(Pp); return ORC_ENOMEM; }
    Pp[0] = NULL;
    if (J >= 1) Pp[1] = Z;

    /* step 1: filtered powers, P_{j+1} = D_tau(Z (x) P_j) (eq. 11) */
    for (int j = 1; j + 1 <= J && rc == ORC_OK; ++j) {
        rc = orc_spgemm(Z, Pp[j], NULL, tau, &P[j + 1], &st, nthreads);
        if (rc == ORC_OK) {
            Pp[j + 1] = &P[j + 1];
            record(stats, max_stats, &ns, &st, 0, j + 1);
        }
    }

    orc_csr S = {0}, T = {0}, Bh = {0};
    if (rc == ORC_OK && b == 1) {
        /* one block only: F = Bhat_0, not filtered (eq. 13) */
        rc = coefficient_block(Pp, c, m, q, 0, q - 1, n, &S, &st, nthreads);
        if (rc == ORC_OK) record(stats, max_stats, &ns, &st, 1, 0);
    } else if (rc == ORC_OK) {
        if (g) {
            /* S_1 = Bhat_{b-2} + c_{(b-1)q} P_q: no product, no filter (eq. 14) */
            rc = coefficient_block(Pp, c, m, q, b - 2, q, n, &S, &st, nthreads);
            if (rc == ORC_OK) record(stats, max_stats, &ns, &st, 2, 1);
        } else {
            /* S_0 = Bhat_{b-1} (eq. 14) */
            rc = coefficient_block(Pp, c, m, q, b - 1, q - 1, n, &S, &st, nthreads);
            if (rc == ORC_OK) record(stats, max_stats, &ns, &st, 1, b - 1);
        }
        /* S_i = D_tau(Bhat_{b-1-i} + P_q (x) S_{i-1}) (eq. 14) */
        for (int i = start; i <= b - 1 && rc == ORC_OK; ++i) {
            rc = coefficient_block(Pp, c, m, q, b - 1 - i, q - 1, n, &Bh, &st, nthreads);
            if (rc != ORC_OK) break;
            record(stats, max_stats, &ns, &st, 1, b - 1 - i);
            rc = orc_spgemm(Pp[q], &S, &Bh, tau, &T, &st, nthreads);
            orc_csr_free(&Bh);
            if (rc != ORC_OK) break;
            record(stats, max_stats, &ns, &st, 3, i);
            orc_csr_free(&S);
            S = T;
            memset(&T, 0, sizeof(T));
        }
    }
    for (int j = 2; j <= J; ++j) orc_csr_free(&P[j]);
    free(P);
    free(Pp);
    if (rc != ORC_OK) {
        orc_csr_free(&S);
        return rc;
    }
    *F = S;
    if (n_stats) *n_stats = ns;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* plain definition, long double: P_m(Z) by Horner (Qin) on dense Z     */
/* ------------------------------------------------------------------ */

/*
 * Y = c_m I; for k = m-1..0: Y = Y Z + c_k I  (eq. 1 evaluated by the Qin /
 * Horner scheme of Section 2.1), in long double on a dense n x n matrix
 * (row-major).  For brute-force checks on small n.
 */
int orc_dense_horner_ld(int64_t n, const double *Zd, const double *c, int m, long double *Y)
{
    if (n < 0 || m < 0 || !Zd || !c || !Y) return ORC_EINVAL;
    long double *T = malloc((size_t)(n * n > 0 ? n * n : 1) * sizeof(long double));
    long double *Zl = malloc((size_t)(n * n > 0 ? n * n : 1) * sizeof(long double));
    if (!T || !Zl) { free(T); free(Zl); return ORC_ENOMEM; }
    for (int64_t i = 0; i < n * n; ++i) Zl[i] = (long double)Zd[i];
    for (int64_t i = 0; i < n * n; ++i) Y[i] = 0.0L;
    for (int64_t i = 0; i < n; ++i) Y[i * n + i] = (long double)c[m];
    for (int k = m - 1; k >= 0; --k) {
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j) {
                long double s = 0.0L;
                for (int64_t t = 0; t < n; ++t) s += Y[i * n + t] * Zl[t * n + j];
                T[i * n + j] = s;
            }
        for (int64_t i = 0; i < n * n; ++i) Y[i] = T[i];
        for (int64_t i = 0; i < n; ++i) Y[i * n + i] += (long double)c[k];
    }
    free(T);
    free(Zl);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Adaptive filter (Algorithm 1) and the thresholds of eqs. 21-28       */
/* ------------------------------------------------------------------ */

/*
 * 1-norm of the candidate matrix {entries with 0 < |x| <= t} of C, with the
 * column sums taken exactly in integers: every |x| contributes
 * ceil(|x| * 2^40 / eps_g), and the largest column sum is returned divided
 * by the same scale.  This is an upper bound of the exact 1-norm (up to one
 * rounding per entry) and does not depend on the summation order.
 */
static double candidate_norm1(const orc_csr *C, double t, double eps_g)
{
    const double s = ldexp(1.0, 40) / eps_g;
    uint64_t *cs = calloc((size_t)(C->n > 0 ? C->n : 1), sizeof(uint64_t));
    if (!cs) return INFINITY;
    for (int64_t r = 0; r < C->n; ++r)
        for (int64_t p = C->row_ptr[r]; p < C->row_ptr[r + 1]; ++p) {
            const double a = fabs(C->val[p]);
            if (a > 0.0 && a <= t) cs[C->col[p]] += (uint64_t)ceil(a * s);
        }
    uint64_t mx = 0;
    for (int64_t c = 0; c < C->n; ++c)
        if (cs[c] > mx) mx = cs[c];
    free(cs);
    return (double)mx / s;
}

typedef struct {
    double eps_g;      /* filtering-norm threshold of this stage */
    double threshold;  /* final entry threshold: entries with |x| <= threshold dropped */
    double dropped;    /* 1-norm of the dropped entries (integer column sums, as above) */
    int32_t iters;     /* Algorithm 1 iterations */
    int32_t pad;
} orc_alg1_stats;

/*
 * Algorithm 1 on C in place: eps_f = eps_g / m_i, candidates are the entries
 * with |x| <= eps_f (the entries above it are "found" and protected), the
 * candidate norm c_{i+1} and m_{i+1} = c_{i+1} / eps_f follow, until
 * c <= eps_g (1 + e_r); the final candidates are dropped.  m_0 = 1; the
 * sentinel c_0 = 1 is taken as "enter the loop" (at least one iteration).
 * eps_g = +inf drops nothing (no bound applies).
 */
int orc_alg1_filter(orc_csr *C, double eps_g, double e_r, int max_iter, orc_alg1_stats *st)
{
    if (!C || !(eps_g > 0.0) || !(e_r >= 0.0) || max_iter < 1) return ORC_EINVAL;
    /* every candidate adds at most 2^40 + 1 (its |x| <= eps_f <= eps_g) to a
     * 64-bit column sum: exact only while a column has fewer than 2^24 entries */
    if (C->n >= ((int64_t)1 << 24)) return ORC_EINVAL;
    orc_alg1_stats s0 = {eps_g, 0.0, 0.0, 0, 0};
    if (isinf(eps_g)) {
        if (st) *st = s0;
        return ORC_OK;
    }
    const double target = eps_g * (1.0 + e_r);
    double m = 1.0, t = 0.0, c = 0.0;
    int it = 0;
    do {
        t = eps_g / m;
        c = candidate_norm1(C, t, eps_g);
        m = c / t;
        ++it;
    } while (c > target && it < max_iter);
    if (c > target) return ORC_EINVAL; /* did not converge */
    /* drop the candidates */
    int64_t w = 0;
    int64_t *rp = C->row_ptr;
    int64_t start = 0;
    for (int64_t r = 0; r < C->n; ++r) {
        const int64_t b = start, e = rp[r + 1];
        start = e;
        rp[r] = w;
        for (int64_t p = b; p < e; ++p) {
            if (fabs(C->val[p]) <= t) continue;
            C->col[w] = C->col[p];
            C->val[w] = C->val[p];
            ++w;
        }
    }
    rp[C->n] = w;
    C->nnz = w;
    s0.threshold = t;
    s0.dropped = c;
    s0.iters = it;
    if (st) *st = s0;
    return ORC_OK;
}

/*
 * Filtering-norm thresholds for the polynomial case (eq. 28): zeta_k for the
 * powers k = 2..q and sigma_j for the Horner steps, from d_k (eq. 24),
 * beta (eq. 21) and the norm bounds of eqs. 25-26.  z[t] >= ||Z^t|| for
 * t = 0..q(b-1).  Sums run in ascending index order with separate
 * multiplications and additions.  M = the number of filtered stages of the
 * schedule (q + b - 2 - g when b >= 2).  A zero d_k is replaced by 1.
 * zeta[0..q] (entries 0, 1 unused) and sigma[0..b-1] are written.
 */
int orc_fnt_thresholds(const double *coef, int m, int s, double eps, const double *z, double *zeta,
                       double *sigma)
{
    int N, q, b, g, J, start, nsp;
    if (orc_schedule(m, s, &N, &q, &b, &g, &J, &start, &nsp)) return ORC_EINVAL;
#define A_(k) (((k) >= 0 && (k) <= m) ? fabs(coef[(k)]) : 0.0)
    double *nb = calloc((size_t)b, sizeof(double));
    double *ns = calloc((size_t)b, sizeof(double));
    if (!nb || !ns) { free(nb); free(ns); return ORC_ENOMEM; }
    for (int i = 0; i < b; ++i) {
        double acc = 0.0;
        for (int j = 0; j < q; ++j) acc = acc + A_(i * q + j) * z[j];
        nb[i] = acc;
    }
    ns[0] = nb[b - 1];
    for (int i = 1; i < b; ++i) ns[i] = nb[b - 1 - i] + z[q] * ns[i - 1];
    const double M = (double)(nsp > 0 ? nsp : 1);
    for (int k = 0; k <= q; ++k) zeta[k] = INFINITY;
    for (int k = 2; k <= q; ++k) {
        double d = 0.0;
        for (int j = 0; j < b; ++j) {
            const int i = b - 1 - j;
            double beta = 0.0;
            if (k < q)
                for (int kk = k; kk < q; ++kk) beta = beta + A_(i * q + kk) * z[kk - k];
            const double sprev = (j >= 1) ? ns[j - 1] : 0.0;
            d = d + z[q * (b - 1 - j)] * (beta + z[q - k] * sprev);
        }
        if (d == 0.0) d = 1.0;
        zeta[k] = eps / (d * M);
    }
    for (int j = 0; j < b; ++j) sigma[j] = eps / (z[q * (b - 1 - j)] * M);
#undef A_
    free(nb);
    free(ns);
    return ORC_OK;
}

/*
 * Filtered PS with the adaptive filter (Algorithm 2 for a polynomial of
 * known degree, eq. 28 thresholds): every sparse product is formed without
 * filtering (exact zeros dropped) and then filtered by Algorithm 1 with
 * eps_g = zeta_{j+1} (powers) or sigma_i (Horner steps).  Stage records as
 * in orc_filtered_ps; alg1[] receives one record per filtered stage.
 */
int orc_filtered_ps_adaptive(const orc_csr *Z, const double *c, int m, int s, double eps, double e_r,
                             const double *z, orc_csr *F, orc_stage_stats *stats, int max_stats, int *n_stats,
                             orc_alg1_stats *alg1, int max_alg1, int *n_alg1, int nthreads)
{
    int N, q, b, g, J, start, nsp;
    if (!Z || !c || !F || !z || !(eps > 0.0) || orc_schedule(m, s, &N, &q, &b, &g, &J, &start, &nsp))
        return ORC_EINVAL;
    if (q > 255) return ORC_EINVAL;
    double *zeta = malloc((size_t)(q + 1) * sizeof(double));
    double *sigma = malloc((size_t)(b + 1) * sizeof(double));
    if (!zeta || !sigma) { free(zeta); free(sigma); return ORC_ENOMEM; }
    int rc = orc_fnt_thresholds(c, m, s, eps, z, zeta, sigma);
    const int64_t n = Z->n;
    int ns = 0, na = 0;
    orc_stage_stats st;
    orc_alg1_stats a1;
    orc_csr *P = calloc((size_t)(J + 2), sizeof(orc_csr));
    const orc_csr **Pp = calloc((size_t)(J + 2), sizeof(orc_csr *));
    if (!P || !Pp) rc = ORC_ENOMEM;
    if (rc == ORC_OK) {
        Pp[0] = NULL;
        if (J >= 1) Pp[1] = Z;
    }
    for (int j = 1; j + 1 <= J && rc == ORC_OK; ++j) {
        rc = orc_spgemm(Z, Pp[j], NULL, 0.0, &P[j + 1], &st, nthreads);
        if (rc == ORC_OK) rc = orc_alg1_filter(&P[j + 1], zeta[j + 1], e_r, 200, &a1);
        if (rc == ORC_OK) {
            Pp[j + 1] = &P[j + 1];
            st.nnz_kept = P[j + 1].nnz;
            record(stats, max_stats, &ns, &st, 0, j + 1);
            if (na < max_alg1) alg1[na] = a1;
            na++;
        }
    }
    orc_csr S = {0}, T = {0}, Bh = {0};
    if (rc == ORC_OK && b == 1) {
        rc = coefficient_block(Pp, c, m, q, 0, q - 1, n, &S, &st, nthreads);
        if (rc == ORC_OK) record(stats, max_stats, &ns, &st, 1, 0);
    } else if (rc == ORC_OK) {
        if (g) {
            rc = coefficient_block(Pp, c, m, q, b - 2, q, n, &S, &st, nthreads);
            if (rc == ORC_OK) record(stats, max_stats, &ns, &st, 2, 1);
        } else {
            rc = coefficient_block(Pp, c, m, q, b - 1, q - 1, n, &S, &st, nthreads);
            if (rc == ORC_OK) record(stats, max_stats, &ns, &st, 1, b - 1);
        }
        for (int i = start; i <= b - 1 && rc == ORC_OK; ++i) {
            rc = coefficient_block(Pp, c, m, q, b - 1 - i, q - 1, n, &Bh, &st, nthreads);
            if (rc != ORC_OK) break;
            record(stats, max_stats, &ns, &st, 1, b - 1 - i);
            rc = orc_spgemm(Pp[q], &S, &Bh, 0.0, &T, &st, nthreads);
            orc_csr_free(&Bh);
            if (rc == ORC_OK) rc = orc_alg1_filter(&T, sigma[i], e_r, 200, &a1);
            if (rc != ORC_OK) break;
            st.nnz_kept = T.nnz;
            record(stats, max_stats, &ns, &st, 3, i);
            if (na < max_alg1) alg1[na] = a1;
            na++;
            orc_csr_free(&S);
            S = T;
            memset(&T, 0, sizeof(T));
        }
    }
    for (int j = 2; j <= J && P; ++j) orc_csr_free(&P[j]);
    free(P);
    free(Pp);
    free(zeta);
    free(sigma);
    if (rc != ORC_OK) {
        orc_csr_free(&S);
        return rc;
    }
    *F = S;
    if (n_stats) *n_stats = ns;
    if (n_alg1) *n_alg1 = na;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Series mode (Section 3.2; Algorithm 2 steps 1-3; eqs. 33-37)         */
/* ------------------------------------------------------------------ */

/* y = Z x: y_r accumulates Z_rk x_k over the stored k of row r in
 * ascending order, one fused multiply-add each, from +0. */
static void spmv(const orc_csr *Z, const double *x, double *y)
{
    for (int64_t r = 0; r < Z->n; ++r) {
        double acc = 0.0;
        for (int64_t p = Z->row_ptr[r]; p < Z->row_ptr[r + 1]; ++p) acc = fma(Z->val[p], x[Z->col[p]], acc);
        y[r] = acc;
    }
}

/* y = Z^T x: y_c accumulates Z_rc x_r over the rows r holding column c in
 * ascending r, one fused multiply-add each, from +0. */
static void spmv_t(const orc_csr *Z, const double *x, double *y)
{
    for (int64_t c = 0; c < Z->n; ++c) y[c] = 0.0;
    for (int64_t r = 0; r < Z->n; ++r)
        for (int64_t p = Z->row_ptr[r]; p < Z->row_ptr[r + 1]; ++p) y[Z->col[p]] = fma(Z->val[p], x[r], y[Z->col[p]]);
}

/* ||y||_1 = sum_i |y_i|, added in ascending index order from +0 (the plain
 * definition of the vector 1-norm, one rounding per addition). */
static double vec_norm1(const double *y, int64_t n)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s = s + fabs(y[i]);
    return s;
}

/* y = A x with A = Z^p (p products with Z), or A^T x = (Z^T)^p x. */
static void apply_power(const orc_csr *Z, int p, int transpose, const double *x, double *y, double *tmp)
{
    const int64_t n = Z->n;
    memcpy(y, x, (size_t)n * sizeof(double));
    for (int i = 0; i < p; ++i) {
        if (transpose)
            spmv_t(Z, y, tmp);
        else
            spmv(Z, y, tmp);
        memcpy(y, tmp, (size_t)n * sizeof(double));
    }
}

/*
 * The block 1-norm estimator of Higham and Tisseur (the algorithm behind
 * normest1, the paper's refs. [16, 17]) with one column (t = 1) and at most
 * itmax = 5 iterations, on A = Z^p applied implicitly.  The start vector is
 * ones/n; sign(0) = +1; among equal largest |(A^T s)_i| the smallest i is
 * taken.  The result est satisfies est <= ||A||_1 and equals ||A v||_1 for
 * the returned unit vector v = e_ind (ind = -1 when the first iterate won).
 * *iters counts the products with A.
 */
int orc_normest1_power(const orc_csr *Z, int p, double *est_out, int64_t *ind_out, int *iters)
{
    if (!Z || p < 0 || !est_out) return ORC_EINVAL;
    const int64_t n = Z->n;
    const int itmax = 5;
    double *x = malloc((size_t)n * sizeof(double));
    double *y = malloc((size_t)n * sizeof(double));
    double *s = malloc((size_t)n * sizeof(double));
    double *s_old = malloc((size_t)n * sizeof(double));
    double *zt = malloc((size_t)n * sizeof(double));
    double *tmp = malloc((size_t)n * sizeof(double));
    if (!x || !y || !s || !s_old || !zt || !tmp) {
        free(x); free(y); free(s); free(s_old); free(zt); free(tmp);
        return ORC_ENOMEM;
    }
    for (int64_t i = 0; i < n; ++i) x[i] = 1.0 / (double)n;
    double est = 0.0, est_old = 0.0;
    int64_t ind = -1, ind_best = -1;
    int k = 0;
    for (k = 1;; ++k) {
        apply_power(Z, p, 0, x, y, tmp);
        est = vec_norm1(y, n);
        if (est > est_old || k == 2) ind_best = ind;
        if (k >= 2 && est <= est_old) {
            est = est_old;
            break;
        }
        est_old = est;
        if (k > itmax) break;
        for (int64_t i = 0; i < n; ++i) s[i] = (y[i] >= 0.0) ? 1.0 : -1.0;
        if (k >= 2) { /* s parallel to s_old: equal up to sign */
            int same = 1, opposite = 1;
            for (int64_t i = 0; i < n; ++i) {
                if (s[i] != s_old[i]) same = 0;
                if (s[i] != -s_old[i]) opposite = 0;
            }
            if (same || opposite) break;
        }
        memcpy(s_old, s, (size_t)n * sizeof(double));
        apply_power(Z, p, 1, s, zt, tmp);
        double hmax = -1.0;
        int64_t imax = 0;
        for (int64_t i = 0; i < n; ++i)
            if (fabs(zt[i]) > hmax) {
                hmax = fabs(zt[i]);
                imax = i;
            }
        if (k >= 2 && hmax == fabs(zt[ind_best])) break;
        ind = imax;
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        x[ind] = 1.0;
    }
    *est_out = est;
    if (ind_out) *ind_out = ind_best;
    if (iters) *iters = k;
    free(x); free(y); free(s); free(s_old); free(zt); free(tmp);
    return ORC_OK;
}

/*
 * Norm bounds of eq. 37: z[0] = 1, z[i] = the estimate of ||Z^i||_1 for
 * 1 <= i <= K (K = 10 in the paper), and z[i] = alpha^i for i > K with
 * alpha = max_{k = ceil(K/2)..K} z[k]^(1/k) (Lemma 1).  z[0..tmax].
 */
int orc_power_norm_bounds(const orc_csr *Z, int K, int tmax, double *z)
{
    if (!Z || K < 2 || (K % 2) != 0 || tmax < 0 || !z) return ORC_EINVAL;
    z[0] = 1.0;
    const int top = tmax < K ? tmax : K;
    for (int i = 1; i <= top; ++i) {
        const int rc = orc_normest1_power(Z, i, &z[i], NULL, NULL);
        if (rc) return rc;
    }
    if (tmax > K) {
        double alpha = 0.0;
        for (int k = (K + 1) / 2; k <= K; ++k) {
            const double r = pow(z[k], 1.0 / (double)k);
            if (r > alpha) alpha = r;
        }
        for (int i = K + 1; i <= tmax; ++i) z[i] = pow(alpha, (double)i);
    }
    return ORC_OK;
}

/*
 * Eq. 34: N = the smallest m with T_m = sum_{i >= m} |a_i| z_i <= eps_tol/2,
 * the series given by its first L coefficients (terms beyond are taken as
 * zero; N = L means they were not enough and is reported as an error).
 * T_m is accumulated from the end: T_L = 0, T_m = T_{m+1} + |a_m| z_m.
 * Algorithm 2 step 3: q = floor(sqrt(N - 1)) (at least 1).  *tail = T_N.
 */
int orc_series_degree(const double *a, int L, const double *z, double eps_tol, int *N_out, int *q_out,
                      double *tail)
{
    if (!a || L < 1 || !z || !(eps_tol > 0.0) || !N_out || !q_out) return ORC_EINVAL;
    double *T = malloc((size_t)(L + 1) * sizeof(double));
    if (!T) return ORC_ENOMEM;
    T[L] = 0.0;
    for (int m = L - 1; m >= 0; --m) T[m] = T[m + 1] + fabs(a[m]) * z[m];
    int N = L;
    for (int m = 1; m <= L; ++m)
        if (T[m] <= 0.5 * eps_tol) {
            N = m;
            break;
        }
    const double tN = T[N];
    free(T);
    if (N >= L) return ORC_EINVAL;
    int q = 0;
    while ((int64_t)(q + 1) * (q + 1) <= (int64_t)(N - 1)) ++q;
    if (q < 1) q = 1;
    *N_out = N;
    *q_out = q;
    if (tail) *tail = tN;
    return ORC_OK;
}
