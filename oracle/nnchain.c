/*
 * FP64 reference for hierarchical agglomerative clustering (HAC) under
 * complete, average (mean Euclidean, "avg-1"), Ward and average with squared
 * Euclidean distances ("avg-2") linkage.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the oracle that the GPU library is
 * checked against. Nothing in the library links, loads or calls it; only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg do. It
 * shares no code, header, table or constant with the GPU path.
 *
 * What it computes (ParChain paper, Sec. 1 and Sec. 2):
 *   * Linkage distances exactly as defined in Table 1:
 *       complete  max over x in A, y in B of ||x - y||
 *       average   (1 / (|A||B|)) * sum over x in A, y in B of ||x - y||
 *       Ward      sqrt( 2|A||B| / (|A|+|B|) * ||mean(A) - mean(B)||^2 )
 *       avg-2     (1 / (|A||B|)) * sum over x in A, y in B of ||x - y||^2,
 *                 in the chain by its closed form of the same row,
 *                 ||mean(A) - mean(B)||^2 + Var(A)/|A| + Var(B)/|B|, where
 *                 Var is the sum of squared deviations from the mean, kept
 *                 per cluster by the merge rule of Sec. 2.1 (multiplied
 *                 through by |A|+|B|, see dist_avgsq and the merge step);
 *                 oracle_linkage evaluates the double sum itself
 *     always in double precision, by direct coordinate differences (never
 *     the ||x||^2 + ||y||^2 - 2 x.y expansion).
 *   * The sequential nearest-neighbour chain algorithm of the introduction:
 *     grow one chain from a terminal cluster by nearest-neighbour steps until
 *     the top two clusters are reciprocal nearest neighbours, merge them,
 *     continue from what is left of the chain. For reducible linkages
 *     (Sec. 2.1) and inputs without ties this yields the same dendrogram as
 *     merging the globally closest pair at every step.
 *   * Cluster identity follows the paper's footnote in Sec. 1: a cluster's ID
 *     is its lowest point index, and nearest-neighbour ties are broken by
 *     that ID (the comparison key is the pair (distance, cluster ID)).
 *   * The chain starts from the active cluster with the lowest ID (the paper
 *     allows any start; fixing it makes runs reproducible).
 *
 * Inputs are float32 points, widened exactly to double. Output rows are in
 * merge order: (node_a, node_b, height, size), leaves are 0..n-1 and the
 * k-th merge creates node n+k.
 *
 * The candidate scan of each nearest-neighbour query is split over OpenMP
 * threads: every candidate's distance is computed independently into its own
 * array entry and the argmin is taken sequentially afterwards, so the result
 * does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_COMPLETE 0
#define ORC_AVERAGE 1
#define ORC_WARD 2
#define ORC_AVGSQ 3

typedef struct {
    int64_t n;
    int d;
    const float *x;
    /* cluster k (indexed by its ID, the lowest point index) */
    int64_t *head, *tail, *next; /* member list: head[k] -> next[] -> -1 */
    int64_t *size;
    int64_t *node;               /* dendrogram node id of the live cluster */
    double *sum;                 /* n*d coordinate sums, Ward and avg-2 */
    double *var;                 /* sum of squared deviations from the mean, avg-2 */
    long long pair_evals;        /* point-pair distance evaluations */
} orc_state;

static inline double sq_dist(const float *x, int d, int64_t p, int64_t q)
{
    double s = 0.0;
    const float *a = x + (size_t)p * d, *b = x + (size_t)q * d;
    for (int k = 0; k < d; ++k) {
        double t = (double)a[k] - (double)b[k];
        s += t * t;
    }
    return s;
}

/* complete linkage: farthest pair, Table 1 first row */
static double dist_complete(const orc_state *s, int64_t A, int64_t B)
{
    double m = 0.0;
    for (int64_t p = s->head[A]; p >= 0; p = s->next[p])
        for (int64_t q = s->head[B]; q >= 0; q = s->next[q]) {
            double v = sq_dist(s->x, s->d, p, q);
            if (v > m) m = v;
        }
    return sqrt(m);
}

/* average linkage with Euclidean distances (avg-1), Table 1 third row.
 * Neumaier-compensated sum in member order, then one division. */
static double dist_average(const orc_state *s, int64_t A, int64_t B)
{
    double sum = 0.0, c = 0.0;
    for (int64_t p = s->head[A]; p >= 0; p = s->next[p])
        for (int64_t q = s->head[B]; q >= 0; q = s->next[q]) {
            double v = sqrt(sq_dist(s->x, s->d, p, q));
            double t = sum + v;
            if (fabs(sum) >= fabs(v)) c += (sum - t) + v;
            else c += (v - t) + sum;
            sum = t;
        }
    return (sum + c) / ((double)s->size[A] * (double)s->size[B]);
}

/* Ward linkage, closed form of Table 1 second row, centroids from FP64 sums */
static double dist_ward(const orc_state *s, int64_t A, int64_t B)
{
    double na = (double)s->size[A], nb = (double)s->size[B];
    double q = 0.0;
    for (int k = 0; k < s->d; ++k) {
        double t = s->sum[(size_t)A * s->d + k] / na - s->sum[(size_t)B * s->d + k] / nb;
        q += t * t;
    }
    double w = (2.0 * na * nb) / (na + nb);
    return sqrt(w * q);
}

/* average linkage with squared Euclidean distances (avg-2), closed form of
 * Table 1 fourth row: ||mean(A) - mean(B)||^2 + Var(A)/|A| + Var(B)/|B|.
 * The two spread terms are added first, so the value does not depend on
 * which cluster asks. */
static double dist_avgsq(const orc_state *s, int64_t A, int64_t B)
{
    double na = (double)s->size[A], nb = (double)s->size[B];
    double q = 0.0;
    for (int k = 0; k < s->d; ++k) {
        double t = s->sum[(size_t)A * s->d + k] / na - s->sum[(size_t)B * s->d + k] / nb;
        q += t * t;
    }
    return q + (s->var[A] / na + s->var[B] / nb);
}

static double dist(const orc_state *s, int linkage, int64_t A, int64_t B)
{
    switch (linkage) {
    case ORC_COMPLETE: return dist_complete(s, A, B);
    case ORC_AVERAGE: return dist_average(s, A, B);
    case ORC_AVGSQ: return dist_avgsq(s, A, B);
    default: return dist_ward(s, A, B);
    }
}

/* Sec. 2.1 merge rule for the spread of A u B, written for Var = sum of
 * squared deviations (the paper's per-point form times |A|+|B|): the mean
 * of the union is the size-weighted mean of the two means, and
 *   Var(A u B) = |A| ||mean(A) - m||^2 + |B| ||mean(B) - m||^2 + Var(A) + Var(B). */
static double merged_var(const orc_state *s, int64_t A, int64_t B)
{
    double na = (double)s->size[A], nb = (double)s->size[B], nu = na + nb;
    double qa = 0.0, qb = 0.0;
    for (int k = 0; k < s->d; ++k) {
        double ma = s->sum[(size_t)A * s->d + k] / na, mb = s->sum[(size_t)B * s->d + k] / nb;
        double m = (na / nu) * ma + (nb / nu) * mb;
        qa += (ma - m) * (ma - m);
        qb += (mb - m) * (mb - m);
    }
    return (na * qa + nb * qb) + (s->var[A] + s->var[B]);
}

/*
 * Sequential NN-chain HAC.
 *   x        n*d float32 points (row-major)
 *   linkage  0 complete, 1 average, 2 Ward, 3 avg-2
 *   nthreads OpenMP threads for the candidate scan (<=0: runtime default)
 *   out_a/out_b/out_h/out_size  n-1 rows in merge order
 *   cert     optional double[4]: [0] min relative gap (d2-d1)/d2 between the
 *            best and second-best candidate over all queries (1 if none),
 *            [1] number of queries whose best distance is exactly 0,
 *            [2] number of nearest-neighbour queries,
 *            [3] number of point-pair distance evaluations (0 for Ward, avg-2)
 * Returns 0 on success, -1 on bad arguments, -3 on allocation failure.
 */
int oracle_nnchain(const float *x, int64_t n, int d, int linkage, int nthreads,
                   int64_t *out_a, int64_t *out_b, double *out_h, int64_t *out_size,
                   double *cert)
{
    if (n < 1 || d < 1 || !x || linkage < 0 || linkage > 3) return -1;
    if (n > 1 && (!out_a || !out_b || !out_h || !out_size)) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    orc_state s;
    memset(&s, 0, sizeof s);
    s.n = n;
    s.d = d;
    s.x = x;
    s.head = malloc(sizeof(int64_t) * n);
    s.tail = malloc(sizeof(int64_t) * n);
    s.next = malloc(sizeof(int64_t) * n);
    s.size = malloc(sizeof(int64_t) * n);
    s.node = malloc(sizeof(int64_t) * n);
    int64_t *act = malloc(sizeof(int64_t) * n);   /* active cluster IDs */
    int64_t *pos = malloc(sizeof(int64_t) * n);   /* ID -> index in act */
    int64_t *chain = malloc(sizeof(int64_t) * n); /* the chain (a stack) */
    double *cand = malloc(sizeof(double) * n);
    const int centroids = linkage == ORC_WARD || linkage == ORC_AVGSQ;
    if (centroids) s.sum = malloc(sizeof(double) * (size_t)n * d);
    if (linkage == ORC_AVGSQ) s.var = calloc((size_t)n, sizeof(double));
    if (!s.head || !s.tail || !s.next || !s.size || !s.node || !act || !pos || !chain || !cand ||
        (centroids && !s.sum) || (linkage == ORC_AVGSQ && !s.var)) {
        free(s.head); free(s.tail); free(s.next); free(s.size); free(s.node);
        free(act); free(pos); free(chain); free(cand); free(s.sum); free(s.var);
        return -3;
    }
    for (int64_t i = 0; i < n; ++i) {
        s.head[i] = s.tail[i] = i;
        s.next[i] = -1;
        s.size[i] = 1;
        s.node[i] = i;
        act[i] = i;
        pos[i] = i;
        if (s.sum)
            for (int k = 0; k < d; ++k) s.sum[(size_t)i * d + k] = (double)x[(size_t)i * d + k];
    }
    int64_t nact = n, depth = 0, nmerge = 0;
    double min_gap = 1.0, zero_best = 0.0, queries = 0.0;
    long long pairs = 0;

    while (nact > 1) {
        if (depth == 0) {
            /* start a new chain at the lowest active ID */
            int64_t lo = act[0];
            for (int64_t i = 1; i < nact; ++i)
                if (act[i] < lo) lo = act[i];
            chain[depth++] = lo;
        }
        const int64_t a = chain[depth - 1];
        /* distances from a to every other active cluster */
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < nact; ++i)
            cand[i] = (act[i] == a) ? INFINITY : dist(&s, linkage, a, act[i]);
        if (!centroids) pairs += (long long)s.size[a] * (long long)(n - s.size[a]);
        queries += 1.0;
        /* argmin over the key (distance, cluster ID); also the runner-up value */
        int64_t b = -1;
        double bd = INFINITY, second = INFINITY;
        for (int64_t i = 0; i < nact; ++i) {
            if (act[i] == a) continue;
            double v = cand[i];
            if (b < 0 || v < bd || (v == bd && act[i] < b)) {
                if (b >= 0) second = bd;
                bd = v;
                b = act[i];
            } else if (v < second) {
                second = v;
            }
        }
        if (bd == 0.0) zero_best += 1.0;
        if (isfinite(second) && second > 0.0) {
            double g = (second - bd) / second;
            if (g < min_gap) min_gap = g;
        }
        if (depth >= 2 && chain[depth - 2] == b) {
            /* reciprocal nearest neighbours: merge a and b */
            depth -= 2;
            int64_t lo = a < b ? a : b, hi = a < b ? b : a;
            out_a[nmerge] = s.node[a] < s.node[b] ? s.node[a] : s.node[b];
            out_b[nmerge] = s.node[a] < s.node[b] ? s.node[b] : s.node[a];
            out_h[nmerge] = bd;
            out_size[nmerge] = s.size[a] + s.size[b];
            /* members of hi appended to lo; spreads merged (from the old
               means), then sums added */
            if (s.var) s.var[lo] = merged_var(&s, lo, hi);
            s.next[s.tail[lo]] = s.head[hi];
            s.tail[lo] = s.tail[hi];
            s.size[lo] += s.size[hi];
            if (s.sum)
                for (int k = 0; k < d; ++k) s.sum[(size_t)lo * d + k] += s.sum[(size_t)hi * d + k];
            s.node[lo] = n + nmerge;
            ++nmerge;
            /* remove hi from the active set */
            int64_t ph = pos[hi], last = act[nact - 1];
            act[ph] = last;
            pos[last] = ph;
            --nact;
        } else {
            chain[depth++] = b;
        }
    }
    if (cert) {
        cert[0] = min_gap;
        cert[1] = zero_best;
        cert[2] = queries;
        cert[3] = (double)pairs;
    }
    free(s.head); free(s.tail); free(s.next); free(s.size); free(s.node);
    free(act); free(pos); free(chain); free(cand); free(s.sum); free(s.var);
    return 0;
}

/*
 * Linkage distance between two explicit member sets, from the Table 1
 * definitions (Ward: centroids from FP64 sums taken in member order; avg-2:
 * the double sum of squared distances, not its closed form).
 * Returns NAN on bad arguments.
 */
double oracle_linkage(const float *x, int d, int linkage, const int64_t *A, int64_t na,
                      const int64_t *B, int64_t nb)
{
    if (!x || d < 1 || !A || !B || na < 1 || nb < 1) return NAN;
    if (linkage == ORC_WARD) {
        double q = 0.0;
        for (int k = 0; k < d; ++k) {
            double sa = 0.0, sb = 0.0;
            for (int64_t i = 0; i < na; ++i) sa += (double)x[(size_t)A[i] * d + k];
            for (int64_t j = 0; j < nb; ++j) sb += (double)x[(size_t)B[j] * d + k];
            double t = sa / (double)na - sb / (double)nb;
            q += t * t;
        }
        double w = (2.0 * (double)na * (double)nb) / ((double)na + (double)nb);
        return sqrt(w * q);
    }
    if (linkage == ORC_COMPLETE) {
        double m = 0.0;
        for (int64_t i = 0; i < na; ++i)
            for (int64_t j = 0; j < nb; ++j) {
                double v = sq_dist(x, d, A[i], B[j]);
                if (v > m) m = v;
            }
        return sqrt(m);
    }
    if (linkage == ORC_AVERAGE || linkage == ORC_AVGSQ) {
        double sum = 0.0, c = 0.0;
        for (int64_t i = 0; i < na; ++i)
            for (int64_t j = 0; j < nb; ++j) {
                double v = sq_dist(x, d, A[i], B[j]);
                if (linkage == ORC_AVERAGE) v = sqrt(v);
                double t = sum + v;
                if (fabs(sum) >= fabs(v)) c += (sum - t) + v;
                else c += (v - t) + sum;
                sum = t;
            }
        return (sum + c) / ((double)na * (double)nb);
    }
    return NAN;
}

/*
 * Coordinate sums and sizes of every node of a dendrogram given as rows
 * (a, b, height, size) in a valid creation order (children before parents,
 * leaves 0..n-1, row r creates node n+r). Used by the tests to recompute
 * Ward distances between arbitrary live clusters at full scale.
 *   sums  (2n-1) x d doubles, sizes (2n-1)
 * Returns 0, or -1 if a row references a node not yet created.
 */
int oracle_tree_sums(const float *x, int64_t n, int d, const double *rows, double *sums, int64_t *sizes)
{
    for (int64_t i = 0; i < n; ++i) {
        sizes[i] = 1;
        for (int k = 0; k < d; ++k) sums[(size_t)i * d + k] = (double)x[(size_t)i * d + k];
    }
    for (int64_t r = 0; r + 1 < n; ++r) {
        int64_t a = (int64_t)rows[4 * r], b = (int64_t)rows[4 * r + 1], c = n + r;
        if (a < 0 || b < 0 || a >= c || b >= c) return -1;
        sizes[c] = sizes[a] + sizes[b];
        for (int k = 0; k < d; ++k)
            sums[(size_t)c * d + k] = sums[(size_t)a * d + k] + sums[(size_t)b * d + k];
    }
    return 0;
}
