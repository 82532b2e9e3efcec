/*
 * ejoin_oracle.c -- FP64 CPU oracle for the context-enhanced similarity join.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * bench's CPU-baseline leg load this library.  It shares no code, header,
 * table or constant with the GPU library and never touches a device.
 *
 * What it computes is the plain definition of the join, written out:
 *
 *  - cosine similarity of two embedding vectors (Section III.A, the
 *    "Cosine Similarity" equation): dot(a,b) / (||a|| ||b||);
 *  - the theta-join as a selection over the Cartesian product of the embedded
 *    relations (Section III.C, the Cartesian-product, theta-join and
 *    E-theta-join equivalences): every ordered pair (i, j) of R x S whose
 *    similarity passes the threshold;
 *  - the result as pairs of tuple offsets (Section IV.C, the mapping of blocks
 *    back to tuple offsets, "late materialisation");
 *  - the top-k join condition used in the scan-versus-probe study
 *    (Section VI.E): per R tuple, the k most similar S tuples.
 *
 * Canonical FP64 similarity ("sim64"), the exact rule every mode of the GPU
 * library must reproduce:
 *
 *    inputs widened float -> double (exact);
 *    dot(a,b) = (((0 + a0*b0) + a1*b1) + ...), k = 0 .. d-1, one rounding for
 *               each product and each sum (no fused multiply-add; this file
 *               is compiled with -ffp-contract=off and without fast-math);
 *    sim64(r,s) = dot(r,s) / sqrt(dot(r,r) * dot(s,s)),
 *    sim64 := 0 when dot(r,r) == 0 or dot(s,s) == 0.
 *
 * The single square root of the product (instead of the equation's product of
 * two roots) makes sim64(x,x) exactly 1 and sim64 bitwise symmetric.  The
 * match predicate is sim64 >= theta (the paper says "larger than the
 * threshold"; the two differ only on exact ties, which this rule makes
 * well defined).
 *
 * Threads split the outer loop over R rows; each pair's sum is still taken in
 * the order above, so the thread count never changes a result.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* sequential dot product in FP64, one rounding per product and per sum */
static double dot_seq(const float *a, const float *b, int d)
{
    double acc = 0.0;
    for (int k = 0; k < d; ++k) {
        double p = (double)a[k] * (double)b[k];
        acc = acc + p;
    }
    return acc;
}

/* canonical similarity from a dot product and the two squared norms */
static double sim_from(double dot, double nr, double ns)
{
    if (nr == 0.0 || ns == 0.0)
        return 0.0;
    return dot / sqrt(nr * ns);
}

static int all_finite(const float *X, int64_t n, int64_t ld, int d)
{
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < d; ++k)
            if (!isfinite(X[i * ld + k]))
                return 0;
    return 1;
}

static void set_threads(int nthreads)
{
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
}

int eo_max_threads(void) { return omp_get_max_threads(); }

/* squared norms, sequential as in dot_seq */
static double *row_norms(const float *X, int64_t n, int64_t ld, int d)
{
    double *nrm = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!nrm)
        return NULL;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        nrm[i] = dot_seq(X + i * ld, X + i * ld, d);
    return nrm;
}

/* sim64 of one pair */
double eo_sim64(const float *r, const float *s, int d)
{
    return sim_from(dot_seq(r, s, d), dot_seq(r, r, d), dot_seq(s, s, d));
}

/* sim64 of a list of (ri[p], si[p]) pairs. Returns 0, or -1 on bad input. */
int eo_sim64_pairs(const float *R, int64_t ldR, const float *S, int64_t ldS,
                   int d, const int64_t *ri, const int64_t *si, int64_t n,
                   double *out, int nthreads)
{
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p)
        out[p] = eo_sim64(R + ri[p] * ldR, S + si[p] * ldS, d);
    return 0;
}

/*
 * Threshold join: all (i, j) with sim64(r_i, s_j) >= theta, in (i, j)
 * ascending order.  The three output arrays are allocated here (malloc) and
 * released with eo_free.  *n_ties receives the number of pairs whose sim64 lies
 * within tie_eps of theta (reported, never used to decide).
 * Returns the pair count, -1 on non-finite input, -2 on allocation failure.
 */
typedef struct { int64_t n, cap; int32_t *j; double *sc; } rowbuf;

static int rowbuf_push(rowbuf *b, int32_t j, double sc)
{
    if (b->n == b->cap) {
        int64_t nc = b->cap ? 2 * b->cap : 16;
        int32_t *nj = (int32_t *)realloc(b->j, sizeof(int32_t) * (size_t)nc);
        if (!nj) return -1;
        b->j = nj;
        double *ns = (double *)realloc(b->sc, sizeof(double) * (size_t)nc);
        if (!ns) return -1;
        b->sc = ns;
        b->cap = nc;
    }
    b->j[b->n] = j; b->sc[b->n] = sc; ++b->n;
    return 0;
}

int64_t eo_threshold(const float *R, int64_t nR, int64_t ldR,
                     const float *S, int64_t nS, int64_t ldS, int d,
                     double theta, int nthreads, double tie_eps,
                     int32_t **out_r, int32_t **out_s, double **out_score,
                     int64_t *n_ties)
{
    *out_r = NULL; *out_s = NULL; *out_score = NULL; *n_ties = 0;
    if (!all_finite(R, nR, ldR, d) || !all_finite(S, nS, ldS, d))
        return -1;
    set_threads(nthreads);
    double *nr = row_norms(R, nR, ldR, d);
    double *ns = row_norms(S, nS, ldS, d);
    rowbuf *rb = (rowbuf *)calloc((size_t)(nR > 0 ? nR : 1), sizeof(rowbuf));
    if (!nr || !ns || !rb) { free(nr); free(ns); free(rb); return -2; }

    int64_t ties = 0, fail = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+:ties, fail)
    for (int64_t i = 0; i < nR; ++i) {
        for (int64_t j = 0; j < nS; ++j) {
            double sim = sim_from(dot_seq(R + i * ldR, S + j * ldS, d), nr[i], ns[j]);
            if (sim >= theta && rowbuf_push(&rb[i], (int32_t)j, sim) != 0) ++fail;
            if (fabs(sim - theta) < tie_eps) ++ties;
        }
    }
    int64_t total = 0;
    for (int64_t i = 0; i < nR; ++i) total += rb[i].n;
    int32_t *orr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
    int32_t *oss = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
    double *osc = (double *)malloc(sizeof(double) * (size_t)(total > 0 ? total : 1));
    if (fail || !orr || !oss || !osc) {
        for (int64_t i = 0; i < nR; ++i) { free(rb[i].j); free(rb[i].sc); }
        free(rb); free(orr); free(oss); free(osc); free(nr); free(ns);
        return -2;
    }
    int64_t w = 0;
    for (int64_t i = 0; i < nR; ++i) {
        for (int64_t p = 0; p < rb[i].n; ++p) {
            orr[w] = (int32_t)i; oss[w] = rb[i].j[p]; osc[w] = rb[i].sc[p]; ++w;
        }
        free(rb[i].j); free(rb[i].sc);
    }
    free(rb); free(nr); free(ns);
    *out_r = orr; *out_s = oss; *out_score = osc; *n_ties = ties;
    return total;
}

/* strict order used by top-k: higher sim first, then smaller index */
static int better(double sa, int64_t ja, double sb, int64_t jb)
{
    return (sa > sb) || (sa == sb && ja < jb);
}

/*
 * Top-k join: for each R row, the first min(k, |S|) S indices in the order
 * (sim64 descending, index ascending); slots beyond |S| hold index -1 and
 * score -inf.  out_idx / out_score are caller-owned, nR * k entries each.
 * Kept by insertion into a sorted list of length k, which yields exactly the
 * first k elements of the full sort.
 * Returns 0, -1 on non-finite input, -2 on allocation failure.
 */
int eo_topk(const float *R, int64_t nR, int64_t ldR,
            const float *S, int64_t nS, int64_t ldS, int d, int k,
            int nthreads, int64_t *out_idx, double *out_score)
{
    if (!all_finite(R, nR, ldR, d) || !all_finite(S, nS, ldS, d))
        return -1;
    set_threads(nthreads);
    double *nr = row_norms(R, nR, ldR, d);
    double *ns = row_norms(S, nS, ldS, d);
    if (!nr || !ns) { free(nr); free(ns); return -2; }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nR; ++i) {
        int64_t *li = out_idx + i * k;
        double *ls = out_score + i * k;
        int len = 0;
        for (int64_t j = 0; j < nS; ++j) {
            double sim = sim_from(dot_seq(R + i * ldR, S + j * ldS, d), nr[i], ns[j]);
            if (len == k && !better(sim, j, ls[k - 1], li[k - 1]))
                continue;
            int pos = (len < k) ? len : k - 1;   /* slot to fill */
            while (pos > 0 && better(sim, j, ls[pos - 1], li[pos - 1])) {
                ls[pos] = ls[pos - 1]; li[pos] = li[pos - 1]; --pos;
            }
            ls[pos] = sim; li[pos] = j;
            if (len < k) ++len;
        }
        for (int p = len; p < k; ++p) { li[p] = -1; ls[p] = -INFINITY; }
    }
    free(nr); free(ns);
    return 0;
}

/* dense FP64 similarity block (for small checks), out is nR x nS row-major */
int eo_sim_matrix(const float *R, int64_t nR, int64_t ldR,
                  const float *S, int64_t nS, int64_t ldS, int d,
                  int nthreads, double *out)
{
    set_threads(nthreads);
    double *nr = row_norms(R, nR, ldR, d);
    double *ns = row_norms(S, nS, ldS, d);
    if (!nr || !ns) { free(nr); free(ns); return -2; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nR; ++i)
        for (int64_t j = 0; j < nS; ++j)
            out[i * nS + j] = sim_from(dot_seq(R + i * ldR, S + j * ldS, d), nr[i], ns[j]);
    free(nr); free(ns);
    return 0;
}

void eo_free(void *p) { free(p); }
