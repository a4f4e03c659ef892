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

/* ======================================================================
 * Accelerated mode: the same sequential NN-chain, with every nearest-
 * neighbour query answered through a uniform grid over cluster centroids
 * and exact pruning by the paper's lower bounds (Sec. 4.1 Ward, Sec. 4.2
 * average, Sec. 4.3 complete; the search radii of Table 1):
 *   Ward      D(A,C) >= sqrt(2|A|m / (|A|+m)) * ||c_A - c_C||, m the
 *             smallest active size (the weight grows with |C|);
 *   avg-2     D(A,C) >= ||c_A - c_C||^2 + Var(A)/|A|;
 *   average   D(A,C) >= ||c_A - c_C|| (the mean of distances is at least
 *             the distance of the means);
 *   complete  D(A,C) >= ||c_A - c_C||, and >= the extent of the two
 *             clusters' tight boxes along any axis (box faces are attained
 *             by real points).
 * Distances in the grid use only its axes (a lower bound of the full
 * centroid distance). A candidate is skipped only when its bound exceeds
 * (1 + 2^-20) times the best value found so far, so every candidate that can
 * win or tie is evaluated, with the same distance functions as plain mode:
 * the rows are bit for bit those of plain mode. Complete linkage evaluates a
 * candidate's farthest pair exactly with two exact shortcuts that cannot
 * change a maximum: points whose farthest possible partner (box corner and
 * enclosing sphere of the other cluster) cannot beat the running maximum are
 * skipped, and a pair already beyond the cut-off ends the evaluation (the
 * candidate then cannot win). Complete values are also memoised by node
 * pair and combined by the Lance-Williams rule of Table 2 for complete
 * linkage, D(A u B, C) = max(D(A,C), D(B,C)), which is exact.
 *
 * Tie certificate: a skipped candidate exceeds the best by more than a
 * relative 2^-21, so plain mode's smallest gap below 2^-23 is found
 * exactly; this mode reports min(plain mode's min_gap, 2^-23).
 * ====================================================================== */
#define ORC_PRUNE (1.0 + 1.0 / 1048576.0) /* 1 + 2^-20 */
#define ORC_GAP_CAP (1.0 / 8388608.0)     /* 2^-23 */
#define ORC_BLK 8                         /* cells per block edge */
#ifndef ORC_CELLS_PER_CLUSTER
#define ORC_CELLS_PER_CLUSTER 2           /* grid cells per active cluster at a (re)build */
#endif

typedef struct {
    int g;            /* grid axes: the first min(d, 3) coordinates */
    double org[3], h, inv_h, eps;
    int64_t G[3];
    int64_t ncell;
    int32_t *head;    /* per cell: first cluster ID in it, -1 if empty */
    int64_t *cmin;    /* per cell: smallest size of a cluster in it */
    /* second level: blocks of ORC_BLK^g cells with their cluster count and
       smallest size (so that empty or far regions are skipped at once) */
    int64_t SG[3], nblk;
    int64_t *bcnt, *bmin;
    const int64_t *size;
    int32_t *nx, *pv; /* per cluster: next / previous cluster in its cell */
    int64_t *cell;    /* per cluster: its cell */
} orc_grid;

typedef struct {
    uint64_t *key; /* 0 = empty; else (lower node << 32 | higher node) + 1 */
    double *val;   /* >= 0: the exact value; < 0: -(a lower bound) */
    uint64_t mask;
    int64_t used;
} orc_memo;

static uint64_t memo_hash(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

static uint64_t memo_key(int64_t u, int64_t v)
{
    uint64_t lo = (uint64_t)(u < v ? u : v), hi = (uint64_t)(u < v ? v : u);
    return ((lo << 32) | hi) + 1u;
}

/* 1: exact value, 2: lower bound, 0: unknown */
static int memo_get(const orc_memo *M, int64_t u, int64_t v, double *out)
{
    if (!M->key) return 0;
    uint64_t k = memo_key(u, v), i = memo_hash(k) & M->mask;
    for (;;) {
        if (M->key[i] == 0) return 0;
        if (M->key[i] == k) {
            double w = M->val[i];
            *out = w >= 0.0 ? w : -w;
            return w >= 0.0 ? 1 : 2;
        }
        i = (i + 1) & M->mask;
    }
}

static void memo_put(orc_memo *M, int64_t u, int64_t v, double w)
{
    if (!M->key) return;
    if (M->used * 2 > (int64_t)M->mask) {
        /* lossy: forget everything (only speed depends on the memo) */
        memset(M->key, 0, sizeof(uint64_t) * (M->mask + 1));
        M->used = 0;
    }
    uint64_t k = memo_key(u, v), i = memo_hash(k) & M->mask;
    for (;;) {
        if (M->key[i] == 0) {
            M->key[i] = k;
            M->val[i] = w;
            ++M->used;
            return;
        }
        if (M->key[i] == k) {
            /* an exact value replaces a bound; a bound never replaces a value */
            if (w >= 0.0 || M->val[i] < 0.0) M->val[i] = w;
            return;
        }
        i = (i + 1) & M->mask;
    }
}

static void grid_cell_coords(const orc_grid *G, const double *c, int64_t *ci)
{
    for (int k = 0; k < G->g; ++k) {
        double f = floor((c[k] - G->org[k]) * G->inv_h);
        int64_t i = f < 0.0 ? 0 : (f >= (double)G->G[k] ? G->G[k] - 1 : (int64_t)f);
        ci[k] = i;
    }
}

static int64_t grid_index(const orc_grid *G, const int64_t *ci)
{
    int64_t idx = 0;
    for (int k = G->g - 1; k >= 0; --k) idx = idx * G->G[k] + ci[k];
    return idx;
}

static int64_t block_of(const orc_grid *G, const int64_t *ci)
{
    int64_t idx = 0;
    for (int k = G->g - 1; k >= 0; --k) idx = idx * G->SG[k] + ci[k] / ORC_BLK;
    return idx;
}

/* smallest size in a block, from its cells' exact values */
static int64_t block_min(const orc_grid *G, int64_t b)
{
    int64_t bc[3], rem = b, ci[3];
    for (int k = 0; k < G->g; ++k) {
        bc[k] = rem % G->SG[k];
        rem /= G->SG[k];
    }
    int64_t m = INT64_MAX, total = 1;
    for (int k = 0; k < G->g; ++k) total *= ORC_BLK;
    for (int64_t it = 0; it < total; ++it) {
        int64_t r2 = it, ok = 1;
        for (int k = 0; k < G->g; ++k) {
            ci[k] = bc[k] * ORC_BLK + r2 % ORC_BLK;
            r2 /= ORC_BLK;
            if (ci[k] >= G->G[k]) ok = 0;
        }
        if (!ok) continue;
        int64_t c = grid_index(G, ci);
        if (G->head[c] >= 0 && G->cmin[c] < m) m = G->cmin[c];
    }
    return m;
}

static void grid_insert(orc_grid *G, int64_t id, const double *c)
{
    int64_t ci[3];
    grid_cell_coords(G, c, ci);
    int64_t cell = grid_index(G, ci);
    const int64_t blk = block_of(G, ci);
    ++G->bcnt[blk];
    if (G->size[id] < G->bmin[blk]) G->bmin[blk] = G->size[id];
    G->cell[id] = cell;
    G->pv[id] = -1;
    G->nx[id] = G->head[cell];
    if (G->head[cell] >= 0) G->pv[G->head[cell]] = (int32_t)id;
    else G->cmin[cell] = INT64_MAX;
    G->head[cell] = (int32_t)id;
    if (G->size[id] < G->cmin[cell]) G->cmin[cell] = G->size[id];
}

static void grid_remove(orc_grid *G, int64_t id)
{
    int64_t cell = G->cell[id];
    if (G->pv[id] >= 0) G->nx[G->pv[id]] = G->nx[id];
    else G->head[cell] = G->nx[id];
    if (G->nx[id] >= 0) G->pv[G->nx[id]] = G->pv[id];
    /* the cell's smallest size, recounted over what is left */
    int64_t m = INT64_MAX;
    for (int32_t c = G->head[cell]; c >= 0; c = G->nx[c])
        if (G->size[c] < m) m = G->size[c];
    G->cmin[cell] = m;
    int64_t ci[3], rem = cell;
    for (int k = 0; k < G->g; ++k) {
        ci[k] = rem % G->G[k];
        rem /= G->G[k];
    }
    const int64_t blk = block_of(G, ci);
    if (--G->bcnt[blk] == 0) G->bmin[blk] = INT64_MAX;
    else G->bmin[blk] = block_min(G, blk);
}

/* (re)build the grid over the active clusters: about two clusters per cell */
static int grid_build(orc_grid *G, const double *lo, const double *hi, const double *cen, int d,
                      const int64_t *act, int64_t nact)
{
    double vol = 1.0;
    int live = 0;
    for (int k = 0; k < G->g; ++k) {
        G->org[k] = lo[k];
        double e = hi[k] - lo[k];
        if (e > 0.0) {
            vol *= e;
            ++live;
        }
    }
    double target = (double)ORC_CELLS_PER_CLUSTER * (double)(nact > 1 ? nact : 1);
    G->h = live ? pow(vol / target, 1.0 / live) : 1.0;
    if (!(G->h > 0.0)) G->h = 1.0;
    G->ncell = 1;
    for (int k = 0; k < G->g; ++k) {
        double e = hi[k] - lo[k];
        int64_t c = e > 0.0 ? (int64_t)ceil(e / G->h) : 1;
        if (c < 1) c = 1;
        if (c > 4 * (int64_t)target + 4) c = 4 * (int64_t)target + 4;
        G->G[k] = c;
        G->ncell *= c;
    }
    G->inv_h = 1.0 / G->h;
    double m = 0.0;
    for (int k = 0; k < G->g; ++k) m = fmax(m, fabs(G->org[k]) + fabs(hi[k]));
    G->eps = 1e-6 * G->h + 1e-12 * m;
    G->nblk = 1;
    for (int k = 0; k < G->g; ++k) {
        G->SG[k] = (G->G[k] + ORC_BLK - 1) / ORC_BLK;
        G->nblk *= G->SG[k];
    }
    free(G->head);
    free(G->cmin);
    free(G->bcnt);
    free(G->bmin);
    G->head = malloc(sizeof(int32_t) * (size_t)G->ncell);
    G->cmin = malloc(sizeof(int64_t) * (size_t)G->ncell);
    G->bcnt = calloc((size_t)G->nblk, sizeof(int64_t));
    G->bmin = malloc(sizeof(int64_t) * (size_t)G->nblk);
    if (!G->head || !G->cmin || !G->bcnt || !G->bmin) return -1;
    for (int64_t i = 0; i < G->ncell; ++i) {
        G->head[i] = -1;
        G->cmin[i] = INT64_MAX;
    }
    for (int64_t i = 0; i < G->nblk; ++i) G->bmin[i] = INT64_MAX;
    for (int64_t i = 0; i < nact; ++i) grid_insert(G, act[i], cen + (size_t)act[i] * d);
    return 0;
}

/* smallest distance (grid axes only) from c to the cell with coordinates ci,
 * made smaller by the rounding slack; edge cells extend outwards */
static double cell_gap(const orc_grid *G, const double *c, const int64_t *ci)
{
    double s = 0.0;
    for (int k = 0; k < G->g; ++k) {
        double lo = ci[k] == 0 ? -INFINITY : G->org[k] + (double)ci[k] * G->h;
        double hi = ci[k] == G->G[k] - 1 ? INFINITY : G->org[k] + (double)(ci[k] + 1) * G->h;
        double t = c[k] < lo ? lo - c[k] : (c[k] > hi ? c[k] - hi : 0.0);
        t -= G->eps;
        if (t > 0.0) s += t * t;
    }
    return sqrt(s);
}

typedef struct {
    int64_t b;       /* best candidate ID (-1: none) */
    double bd;       /* its value */
    double second;   /* smallest value among the other evaluated candidates */
} orc_top2;

static void top2_consider(orc_top2 *t, int64_t id, double v)
{
    /* the same update as plain mode's scan */
    if (t->b < 0 || v < t->bd || (v == t->bd && id < t->b)) {
        if (t->b >= 0) t->second = t->bd;
        t->bd = v;
        t->b = id;
    } else if (v < t->second) {
        t->second = v;
    }
}

static double top2_cut(const orc_top2 *t) { return t->b < 0 ? INFINITY : t->bd * ORC_PRUNE; }

typedef struct {
    orc_state s;
    int linkage;
    double *cen;       /* centroids (sum / size), every linkage */
    float *blo, *bhi;  /* complete: tight boxes */
    double *rad;       /* complete: radius of an enclosing sphere about the centroid */
    int64_t *row_a, *row_b; /* node -> children (internal nodes) */
    orc_memo memo;
    float *buf;        /* one cluster's member coordinates, in member order */
    int64_t *idx;      /* one cluster's member indices */
    long long pair_evals, cand_evals;
} orc_fast;

/* copy C's member coordinates, in member-list order, into F->buf */
static const float *gather_members(orc_fast *F, int64_t C)
{
    const int d = F->s.d;
    float *o = F->buf;
    for (int64_t q = F->s.head[C]; q >= 0; q = F->s.next[q]) {
        memcpy(o, F->s.x + (size_t)q * d, sizeof(float) * d);
        o += d;
    }
    return F->buf;
}

/* sq_dist between point p and the j-th gathered point: the same operations
 * in the same order, so the same value */
static inline double sq_dist_buf(const float *x, int d, int64_t p, const float *b)
{
    double s = 0.0;
    const float *a = x + (size_t)p * d;
    for (int k = 0; k < d; ++k) {
        double t = (double)a[k] - (double)b[k];
        s += t * t;
    }
    return s;
}

/* squared distance from point p to the farthest corner of C's box, computed
 * with the same operations as sq_dist (so it bounds every computed sq_dist
 * from p to a member of C, each operation being monotone) */
static double far_corner_sq(const orc_fast *F, int64_t p, int64_t C)
{
    const int d = F->s.d;
    const float *xp = F->s.x + (size_t)p * d;
    const float *lo = F->blo + (size_t)C * d, *hi = F->bhi + (size_t)C * d;
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
        double a = (double)xp[k] - (double)lo[k], b = (double)xp[k] - (double)hi[k];
        double t = fabs(a) > fabs(b) ? a : b;
        s += t * t;
    }
    return s;
}

static double far_sphere_sq(const orc_fast *F, int64_t p, int64_t C)
{
    const int d = F->s.d;
    const float *xp = F->s.x + (size_t)p * d;
    const double *c = F->cen + (size_t)C * d;
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
        double t = (double)xp[k] - c[k];
        s += t * t;
    }
    double r = sqrt(s) * (1.0 + 1e-12) + F->rad[C];
    return r * r * (1.0 + 1e-12);
}

/* complete linkage between A and C: the exact maximum squared point distance
 * (as dist_complete computes it) if it is at most cut2, else a value > cut2
 * with *over = 1 (the evaluation stops at the first pair beyond cut2) */
static double comp_sq_cut(orc_fast *F, int64_t A, int64_t C, double cut2, int *over)
{
    orc_state *s = &F->s;
    const int d = s->d;
    *over = 0;
    /* start from a real pair found by two farthest-point steps */
    int64_t pa = s->head[A];
    double best = -1.0;
    for (int64_t p = s->head[A]; p >= 0; p = s->next[p]) {
        double v = 0.0;
        const float *xp = s->x + (size_t)p * d;
        const double *c = F->cen + (size_t)C * d;
        for (int k = 0; k < d; ++k) {
            double t = (double)xp[k] - c[k];
            v += t * t;
        }
        if (v > best) {
            best = v;
            pa = p;
        }
    }
    const float *cb = gather_members(F, C);
    const int64_t nc = s->size[C];
    double m = -1.0;
    for (int64_t j = 0; j < nc; ++j) {
        double v = sq_dist_buf(s->x, d, pa, cb + (size_t)j * d);
        if (v > m) m = v;
    }
    F->pair_evals += nc;
    if (m > cut2) {
        *over = 1;
        return m;
    }
    const int64_t na = s->size[A];
    if ((double)na * (double)nc < 16384.0) {
        for (int64_t p = s->head[A]; p >= 0; p = s->next[p]) {
            double ub = far_corner_sq(F, p, C);
            double us = far_sphere_sq(F, p, C);
            if (us < ub) ub = us;
            if (ub <= m) continue;
            for (int64_t j = 0; j < nc; ++j) {
                double v = sq_dist_buf(s->x, d, p, cb + (size_t)j * d);
                if (v > m) m = v;
            }
            F->pair_evals += nc;
            if (m > cut2) {
                *over = 1;
                return m;
            }
        }
        return m;
    }
    /* large pairs: the rows of A over threads; a maximum does not depend on
       the order its terms are taken in, and a row is skipped only when it
       cannot exceed the running maximum of its own thread */
    int64_t *rows = F->idx, k = 0;
    for (int64_t p = s->head[A]; p >= 0; p = s->next[p]) rows[k++] = p;
    const double m0 = m;
    int stop = 0;
    long long evals = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(max : m) reduction(+ : evals)
    for (int64_t i = 0; i < na; ++i) {
        int st;
#pragma omp atomic read
        st = stop;
        if (st) continue;
        const int64_t p = rows[i];
        double mm = m > m0 ? m : m0;
        double ub = far_corner_sq(F, p, C);
        double us = far_sphere_sq(F, p, C);
        if (us < ub) ub = us;
        if (ub <= mm) continue;
        for (int64_t j = 0; j < nc; ++j) {
            double v = sq_dist_buf(s->x, d, p, cb + (size_t)j * d);
            if (v > mm) mm = v;
        }
        evals += nc;
        if (mm > m) m = mm;
        if (mm > cut2) {
#pragma omp atomic write
            stop = 1;
        }
    }
    F->pair_evals += evals;
    if (m0 > m) m = m0;
    if (m > cut2) *over = 1;
    return m;
}

/* average linkage as dist_average computes it, stopping (with *over = 1)
 * once the partial mean already exceeds cut */
static double avg_cut(orc_fast *F, int64_t A, int64_t B, double cut, int *over)
{
    const orc_state *s = &F->s;
    double sum = 0.0, c = 0.0;
    const double den = (double)s->size[A] * (double)s->size[B];
    const double lim = cut * den * (1.0 + 1e-9);
    const float *bb = gather_members(F, B);
    const int64_t nb = s->size[B];
    *over = 0;
    for (int64_t p = s->head[A]; p >= 0; p = s->next[p]) {
        for (int64_t j = 0; j < nb; ++j) {
            double v = sqrt(sq_dist_buf(s->x, s->d, p, bb + (size_t)j * s->d));
            double t = sum + v;
            if (fabs(sum) >= fabs(v)) c += (sum - t) + v;
            else c += (v - t) + sum;
            sum = t;
        }
        F->pair_evals += nb;
        if (sum + c > lim) {
            *over = 1;
            return INFINITY;
        }
    }
    return (sum + c) / den;
}

/* complete value through the memo and the Lance-Williams max rule; returns
 * 1 with the exact value, 2 if it is known to exceed cut, 0 if unknown */
static int comp_known(const orc_fast *F, int64_t A, int64_t C, double cut, double *v)
{
    const int64_t n = F->s.n;
    const int64_t na = F->s.node[A], nc = F->s.node[C];
    double w;
    int r = memo_get(&F->memo, na, nc, &w);
    if (r == 1) {
        *v = w;
        return 1;
    }
    if (r == 2 && w > cut) return 2;
    for (int side = 0; side < 2; ++side) {
        int64_t x = side ? nc : na, y = side ? na : nc;
        if (x < n) continue;
        double w1, w2;
        int r1 = memo_get(&F->memo, F->row_a[x - n], y, &w1);
        int r2 = memo_get(&F->memo, F->row_b[x - n], y, &w2);
        if ((r1 && w1 > cut) || (r2 && w2 > cut)) return 2;
        if (r1 == 1 && r2 == 1) {
            *v = w1 > w2 ? w1 : w2;
            return 1;
        }
    }
    return 0;
}

/* lower bound of the linkage value of a cluster whose centroid lies at
 * distance D (grid axes) from A's centroid */
static double lb_of_D(const orc_fast *F, int64_t A, double D, int64_t nmin)
{
    const orc_state *s = &F->s;
    switch (F->linkage) {
    case ORC_WARD: {
        double na = (double)s->size[A], m = (double)nmin;
        return sqrt((2.0 * na * m) / (na + m)) * D;
    }
    case ORC_AVGSQ: return D * D + s->var[A] / (double)s->size[A];
    default: return D;
    }
}

/* evaluate candidate C for query A, unless a bound shows it cannot matter */
static void fast_candidate(orc_fast *F, orc_top2 *t, int64_t A, int64_t C)
{
    orc_state *s = &F->s;
    const int d = s->d;
    const double cut = top2_cut(t);
    ++F->cand_evals;
    if (F->linkage == ORC_WARD || F->linkage == ORC_AVGSQ) {
        top2_consider(t, C, dist(s, F->linkage, A, C));
        return;
    }
    /* centroid distance over all axes */
    const double *ca = F->cen + (size_t)A * d, *cc = F->cen + (size_t)C * d;
    double q = 0.0;
    for (int k = 0; k < d; ++k) {
        double u = ca[k] - cc[k];
        q += u * u;
    }
    double lb = sqrt(q);
    if (F->linkage == ORC_COMPLETE) {
        const float *la = F->blo + (size_t)A * d, *ha = F->bhi + (size_t)A * d;
        const float *lc = F->blo + (size_t)C * d, *hc = F->bhi + (size_t)C * d;
        for (int k = 0; k < d; ++k) {
            double e1 = (double)hc[k] - (double)la[k], e2 = (double)ha[k] - (double)lc[k];
            if (e1 > lb) lb = e1;
            if (e2 > lb) lb = e2;
        }
    }
    if (lb * (1.0 - 1e-12) > cut) return;
    if (F->linkage == ORC_AVERAGE) {
        int over = 0;
        double v = avg_cut(F, A, C, cut, &over);
        if (!over) top2_consider(t, C, v);
        return;
    }
    double v;
    int known = comp_known(F, A, C, cut, &v);
    if (known == 2) return;
    if (known == 0) {
        int over = 0;
        double cut2 = isinf(cut) ? INFINITY : cut * cut;
        double m = comp_sq_cut(F, A, C, cut2, &over);
        if (over) {
            /* D(A,C) > cut (up to rounding): keep a slightly smaller bound */
            if ((double)s->size[A] * (double)s->size[C] >= 64.0)
                memo_put(&F->memo, s->node[A], s->node[C], -cut * (1.0 - 1e-12));
            return;
        }
        v = sqrt(m);
        if ((double)s->size[A] * (double)s->size[C] >= 64.0) memo_put(&F->memo, s->node[A], s->node[C], v);
    }
    top2_consider(t, C, v);
}

/* offsets of the it-th cell (or block) at Chebyshev distance r from a
 * centre, each once over it < shell_count(g, r, k) and k < g: axis k is the
 * first axis at offset +-r, axes before it lie strictly inside, axes after
 * it anywhere in [-r, r] */
static int64_t shell_count(int g, int64_t r, int k)
{
    if (r == 0) return k == 0 ? 1 : 0;
    int64_t total = 2;
    for (int j = 0; j < g; ++j)
        if (j != k) total *= j < k ? 2 * r - 1 : 2 * r + 1;
    return total;
}

static void shell_offset(int g, int64_t r, int k, int64_t it, int64_t *o)
{
    for (int j = 0; j < g; ++j) {
        if (r == 0) {
            o[j] = 0;
        } else if (j == k) {
            o[j] = (it % 2) ? r : -r;
            it /= 2;
        } else {
            const int64_t span = j < k ? 2 * r - 1 : 2 * r + 1;
            o[j] = it % span - (j < k ? r - 1 : r);
            it /= span;
        }
    }
}

static void visit_cell(orc_fast *F, const orc_grid *G, orc_top2 *t, int64_t A, int64_t pre, const double *ca,
                       const int64_t *ci)
{
    const int64_t cell = grid_index(G, ci);
    if (G->head[cell] < 0) return;
    if (lb_of_D(F, A, cell_gap(G, ca, ci), G->cmin[cell]) * (1.0 - 1e-12) > top2_cut(t)) return;
    for (int32_t C = G->head[cell]; C >= 0; C = G->nx[C])
        if (C != A && C != pre) fast_candidate(F, t, A, C);
}

/* nearest-neighbour query of A (key (value, ID)), with the runner-up value
 * among the evaluated candidates; pre: a candidate evaluated first (-1).
 * Cells are visited ring by ring around A's cell up to ORC_BLK rings (so the
 * bound tightens early), then block by block further out. */
static void fast_query(orc_fast *F, orc_grid *G, orc_top2 *t, int64_t A, int64_t pre, int64_t nmin)
{
    t->b = -1;
    t->bd = INFINITY;
    t->second = INFINITY;
    if (pre >= 0) fast_candidate(F, t, A, pre);
    const int g = G->g;
    const double *ca = F->cen + (size_t)A * F->s.d;
    int64_t home[3], ci[3], o[3];
    grid_cell_coords(G, ca, home);
    /* phase 1: cell rings */
    int64_t rmax = 0;
    for (int k = 0; k < g; ++k) {
        int64_t e = home[k] > G->G[k] - 1 - home[k] ? home[k] : G->G[k] - 1 - home[k];
        if (e > rmax) rmax = e;
    }
    const int64_t R1 = rmax < ORC_BLK ? rmax : ORC_BLK;
    for (int64_t r = 0; r <= R1; ++r) {
        double Dr = r == 0 ? 0.0 : (double)(r - 1) * G->h - G->eps;
        if (Dr < 0.0) Dr = 0.0;
        if (lb_of_D(F, A, Dr, nmin) * (1.0 - 1e-12) > top2_cut(t)) return;
        for (int k = 0; k < g; ++k)
            for (int64_t it = 0, cnt = shell_count(g, r, k); it < cnt; ++it) {
                shell_offset(g, r, k, it, o);
                int inside = 1;
                for (int j = 0; j < g; ++j) {
                    ci[j] = home[j] + o[j];
                    if (ci[j] < 0 || ci[j] >= G->G[j]) inside = 0;
                }
                if (inside) visit_cell(F, G, t, A, pre, ca, ci);
            }
    }
    if (R1 == rmax) return;
    /* phase 2: rings of blocks, skipping the cells phase 1 visited */
    int64_t hb[3], bc[3], bmax = 0;
    for (int k = 0; k < g; ++k) {
        hb[k] = home[k] / ORC_BLK;
        int64_t e = hb[k] > G->SG[k] - 1 - hb[k] ? hb[k] : G->SG[k] - 1 - hb[k];
        if (e > bmax) bmax = e;
    }
    const double bh = G->h * ORC_BLK;
    int64_t cells_per_blk = 1;
    for (int k = 0; k < g; ++k) cells_per_blk *= ORC_BLK;
    for (int64_t r = 0; r <= bmax; ++r) {
        double Dr = r == 0 ? 0.0 : (double)(r - 1) * bh - G->eps;
        if (Dr < 0.0) Dr = 0.0;
        if (lb_of_D(F, A, Dr, nmin) * (1.0 - 1e-12) > top2_cut(t)) break;
        for (int k = 0; k < g; ++k)
            for (int64_t it = 0, cnt = shell_count(g, r, k); it < cnt; ++it) {
                shell_offset(g, r, k, it, o);
                int inside = 1;
                for (int j = 0; j < g; ++j) {
                    bc[j] = hb[j] + o[j];
                    if (bc[j] < 0 || bc[j] >= G->SG[j]) inside = 0;
                }
                if (!inside) continue;
                int64_t blk = 0;
                for (int j = g - 1; j >= 0; --j) blk = blk * G->SG[j] + bc[j];
                if (G->bcnt[blk] == 0) continue;
                /* gap to the block's box */
                double q = 0.0;
                for (int j = 0; j < g; ++j) {
                    double lo = bc[j] == 0 ? -INFINITY : G->org[j] + (double)(bc[j] * ORC_BLK) * G->h;
                    double hi = bc[j] == G->SG[j] - 1 ? INFINITY
                                                       : G->org[j] + (double)((bc[j] + 1) * ORC_BLK) * G->h;
                    double u = ca[j] < lo ? lo - ca[j] : (ca[j] > hi ? ca[j] - hi : 0.0);
                    u -= G->eps;
                    if (u > 0.0) q += u * u;
                }
                if (lb_of_D(F, A, sqrt(q), G->bmin[blk]) * (1.0 - 1e-12) > top2_cut(t)) continue;
                for (int64_t c2 = 0; c2 < cells_per_blk; ++c2) {
                    int64_t r2 = c2, ok = 1, far = 0;
                    for (int j = 0; j < g; ++j) {
                        ci[j] = bc[j] * ORC_BLK + r2 % ORC_BLK;
                        r2 /= ORC_BLK;
                        if (ci[j] >= G->G[j]) ok = 0;
                        const int64_t dj = ci[j] > home[j] ? ci[j] - home[j] : home[j] - ci[j];
                        if (dj > R1) far = 1;
                    }
                    if (ok && far) visit_cell(F, G, t, A, pre, ca, ci);
                }
            }
    }
}

/*
 * Accelerated sequential NN-chain HAC: the same chain as oracle_nnchain,
 * with grid-pruned queries (see above). Same arguments and rows; cert is a
 * double[6]: [0] min(min_gap of plain mode, 2^-23), [1] zero-distance bests,
 * [2] queries, [3] point-pair distances evaluated (complete, average),
 * [4] candidate clusters examined, [5] grid rebuilds.
 */
int oracle_nnchain_grid(const float *x, int64_t n, int d, int linkage, int64_t *out_a, int64_t *out_b,
                        double *out_h, int64_t *out_size, double *cert)
{
    if (n < 1 || d < 1 || !x || linkage < 0 || linkage > 3) return -1;
    if (n > 2147483646LL) return -1;
    if (n > 1 && (!out_a || !out_b || !out_h || !out_size)) return -1;
    orc_fast F;
    memset(&F, 0, sizeof F);
    orc_state *s = &F.s;
    F.linkage = linkage;
    s->n = n;
    s->d = d;
    s->x = x;
    orc_grid G;
    memset(&G, 0, sizeof G);
    G.g = d < 3 ? d : 3;
    const int comp = linkage == ORC_COMPLETE;
    s->head = malloc(sizeof(int64_t) * n);
    s->tail = malloc(sizeof(int64_t) * n);
    s->next = malloc(sizeof(int64_t) * n);
    s->size = malloc(sizeof(int64_t) * n);
    s->node = malloc(sizeof(int64_t) * n);
    s->sum = malloc(sizeof(double) * (size_t)n * d);
    if (linkage == ORC_AVGSQ) s->var = calloc((size_t)n, sizeof(double));
    F.cen = malloc(sizeof(double) * (size_t)n * d);
    F.buf = malloc(sizeof(float) * (size_t)n * d);
    F.idx = malloc(sizeof(int64_t) * (size_t)n);
    F.row_a = malloc(sizeof(int64_t) * (size_t)(n > 1 ? n - 1 : 1));
    F.row_b = malloc(sizeof(int64_t) * (size_t)(n > 1 ? n - 1 : 1));
    if (comp) {
        F.blo = malloc(sizeof(float) * (size_t)n * d);
        F.bhi = malloc(sizeof(float) * (size_t)n * d);
        F.rad = calloc((size_t)n, sizeof(double));
        uint64_t cap = 1u << 16;
        while (cap < 4 * (uint64_t)n && cap < (1ull << 26)) cap <<= 1;
        F.memo.key = calloc(cap, sizeof(uint64_t));
        F.memo.val = malloc(sizeof(double) * cap);
        F.memo.mask = cap - 1;
    }
    int64_t *act = malloc(sizeof(int64_t) * n), *pos = malloc(sizeof(int64_t) * n);
    int64_t *chain = malloc(sizeof(int64_t) * n);
    int64_t *scnt = calloc((size_t)n + 1, sizeof(int64_t)); /* clusters of each size */
    G.nx = malloc(sizeof(int32_t) * n);
    G.pv = malloc(sizeof(int32_t) * n);
    G.cell = malloc(sizeof(int64_t) * n);
    int rc = 0;
    if (!s->head || !s->tail || !s->next || !s->size || !s->node || !s->sum || !F.cen || !F.buf || !F.idx || !F.row_a ||
        !F.row_b || (linkage == ORC_AVGSQ && !s->var) ||
        (comp && (!F.blo || !F.bhi || !F.rad || !F.memo.key || !F.memo.val)) || !act || !pos || !chain ||
        !scnt || !G.nx || !G.pv || !G.cell) {
        rc = -3;
        goto done;
    }
    double blo[3] = {INFINITY, INFINITY, INFINITY}, bhi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < n; ++i) {
        s->head[i] = s->tail[i] = i;
        s->next[i] = -1;
        s->size[i] = 1;
        s->node[i] = i;
        act[i] = i;
        pos[i] = i;
        for (int k = 0; k < d; ++k) {
            double v = (double)x[(size_t)i * d + k];
            s->sum[(size_t)i * d + k] = v;
            F.cen[(size_t)i * d + k] = v;
            if (comp) F.blo[(size_t)i * d + k] = F.bhi[(size_t)i * d + k] = x[(size_t)i * d + k];
            if (k < G.g) {
                if (v < blo[k]) blo[k] = v;
                if (v > bhi[k]) bhi[k] = v;
            }
        }
    }
    scnt[1] = n;
    int64_t nmin = 1;
    G.size = s->size;
    if (grid_build(&G, blo, bhi, F.cen, d, act, n) != 0) {
        rc = -3;
        goto done;
    }
    int64_t nact = n, depth = 0, nmerge = 0, lowest = 0, rebuilds = 0;
    double min_gap = 1.0, zero_best = 0.0, queries = 0.0;
    orc_top2 t;
    while (nact > 1) {
        if (depth == 0) {
            while (s->size[lowest] == 0) ++lowest; /* lowest active ID */
            chain[depth++] = lowest;
        }
        const int64_t a = chain[depth - 1];
        const int64_t pre = depth >= 2 ? chain[depth - 2] : -1;
        fast_query(&F, &G, &t, a, pre, nmin);
        queries += 1.0;
        const int64_t b = t.b;
        const double bd = t.bd;
        if (b < 0) {
            rc = -2;
            goto done;
        }
        if (bd == 0.0) zero_best += 1.0;
        if (isfinite(t.second) && t.second > 0.0) {
            double gp = (t.second - bd) / t.second;
            if (gp > ORC_GAP_CAP) gp = ORC_GAP_CAP;
            if (gp < min_gap) min_gap = gp;
        } else if (!isfinite(t.second) && nact >= 3) {
            if (ORC_GAP_CAP < min_gap) min_gap = ORC_GAP_CAP;
        }
        if (pre == b) {
            depth -= 2;
            int64_t lo = a < b ? a : b, hi = a < b ? b : a;
            out_a[nmerge] = s->node[a] < s->node[b] ? s->node[a] : s->node[b];
            out_b[nmerge] = s->node[a] < s->node[b] ? s->node[b] : s->node[a];
            out_h[nmerge] = bd;
            out_size[nmerge] = s->size[a] + s->size[b];
            F.row_a[nmerge] = s->node[lo];
            F.row_b[nmerge] = s->node[hi];
            grid_remove(&G, lo);
            grid_remove(&G, hi);
            if (s->var) s->var[lo] = merged_var(s, lo, hi);
            const int64_t sl = s->size[lo], sh = s->size[hi];
            s->next[s->tail[lo]] = s->head[hi];
            s->tail[lo] = s->tail[hi];
            s->size[lo] = sl + sh;
            s->size[hi] = 0;
            const double nu = (double)(sl + sh);
            double dl = 0.0, dh = 0.0;
            for (int k = 0; k < d; ++k) {
                const size_t il = (size_t)lo * d + k, ih = (size_t)hi * d + k;
                s->sum[il] += s->sum[ih];
                const double c = s->sum[il] / nu;
                dl += (c - F.cen[il]) * (c - F.cen[il]);
                dh += (c - F.cen[ih]) * (c - F.cen[ih]);
                F.cen[il] = c;
                if (comp) {
                    if (F.blo[ih] < F.blo[il]) F.blo[il] = F.blo[ih];
                    if (F.bhi[ih] > F.bhi[il]) F.bhi[il] = F.bhi[ih];
                }
            }
            if (comp) {
                double r1 = sqrt(dl) * (1.0 + 1e-12) + F.rad[lo], r2 = sqrt(dh) * (1.0 + 1e-12) + F.rad[hi];
                F.rad[lo] = (r1 > r2 ? r1 : r2) * (1.0 + 1e-12);
            }
            s->node[lo] = n + nmerge;
            ++nmerge;
            --scnt[sl];
            --scnt[sh];
            ++scnt[sl + sh];
            while (nmin <= n && scnt[nmin] == 0) ++nmin;
            int64_t ph = pos[hi], last = act[nact - 1];
            act[ph] = last;
            pos[last] = ph;
            --nact;
            if (nact > 1 && (double)G.ncell > 8.0 * ORC_CELLS_PER_CLUSTER * (double)nact && G.ncell > 64) {
                if (grid_build(&G, blo, bhi, F.cen, d, act, nact) != 0) {
                    rc = -3;
                    goto done;
                }
                ++rebuilds;
            } else {
                grid_insert(&G, lo, F.cen + (size_t)lo * d);
            }
        } else {
            chain[depth++] = b;
        }
    }
    if (cert) {
        cert[0] = min_gap;
        cert[1] = zero_best;
        cert[2] = queries;
        cert[3] = (double)F.pair_evals;
        cert[4] = (double)F.cand_evals;
        cert[5] = (double)rebuilds;
    }
done:
    free(s->head); free(s->tail); free(s->next); free(s->size); free(s->node); free(s->sum); free(s->var);
    free(F.cen); free(F.buf); free(F.idx); free(F.blo); free(F.bhi); free(F.rad); free(F.row_a); free(F.row_b);
    free(F.memo.key); free(F.memo.val);
    free(act); free(pos); free(chain); free(scnt);
    free(G.nx); free(G.pv); free(G.cell); free(G.head); free(G.cmin); free(G.bcnt); free(G.bmin);
    return rc;
}

/*
 * The dendrogram row convention of the library's output, for large row
 * counts (the tests pin it to the plain Python statement of the same rule):
 * rows sorted by (largest height in the row's subtree, size, lowest point
 * index of the new cluster), children relabelled so that row r creates node
 * n+r, and a < b in every row. rows_in: n-1 rows (a, b, height, size) in a
 * valid creation order; rows_out: n-1 rows. Returns 0, or -1 on a row that
 * references a node not yet created, -3 on allocation failure.
 */
typedef struct {
    double eff;
    int64_t size, lo, r;
} orc_rowkey;

static int rowkey_cmp(const void *pa, const void *pb)
{
    const orc_rowkey *a = pa, *b = pb;
    if (a->eff != b->eff) return a->eff < b->eff ? -1 : 1;
    if (a->size != b->size) return a->size < b->size ? -1 : 1;
    if (a->lo != b->lo) return a->lo < b->lo ? -1 : 1;
    return 0;
}

int oracle_canonical(const double *rows_in, int64_t n, double *rows_out)
{
    const int64_t m = n - 1;
    if (m <= 0) return 0;
    int64_t *lo = malloc(sizeof(int64_t) * (size_t)(2 * n - 1));
    double *eff = malloc(sizeof(double) * (size_t)(2 * n - 1));
    int64_t *newid = malloc(sizeof(int64_t) * (size_t)(2 * n - 1));
    orc_rowkey *key = malloc(sizeof(orc_rowkey) * (size_t)m);
    if (!lo || !eff || !newid || !key) {
        free(lo); free(eff); free(newid); free(key);
        return -3;
    }
    for (int64_t i = 0; i < n; ++i) {
        lo[i] = i;
        eff[i] = 0.0;
        newid[i] = i;
    }
    int rc = 0;
    for (int64_t r = 0; r < m; ++r) {
        int64_t a = (int64_t)rows_in[4 * r], b = (int64_t)rows_in[4 * r + 1];
        if (a < 0 || b < 0 || a >= n + r || b >= n + r) {
            rc = -1;
            break;
        }
        lo[n + r] = lo[a] < lo[b] ? lo[a] : lo[b];
        double e = rows_in[4 * r + 2];
        if (eff[a] > e) e = eff[a];
        if (eff[b] > e) e = eff[b];
        eff[n + r] = e;
        key[r].eff = e;
        key[r].size = (int64_t)rows_in[4 * r + 3];
        key[r].lo = lo[n + r];
        key[r].r = r;
    }
    if (rc == 0) {
        qsort(key, (size_t)m, sizeof(orc_rowkey), rowkey_cmp);
        for (int64_t p = 0; p < m; ++p) newid[n + key[p].r] = n + p;
        for (int64_t p = 0; p < m; ++p) {
            const double *in = rows_in + 4 * key[p].r;
            int64_t a = newid[(int64_t)in[0]], b = newid[(int64_t)in[1]];
            rows_out[4 * p] = (double)(a < b ? a : b);
            rows_out[4 * p + 1] = (double)(a < b ? b : a);
            rows_out[4 * p + 2] = in[2];
            rows_out[4 * p + 3] = in[3];
        }
    }
    free(lo); free(eff); free(newid); free(key);
    return rc;
}

/*
 * Identity of every merge, independent of row order: for each row, the two
 * children as (lowest point index, size) pairs, the smaller pair first.
 * rows: n-1 rows in a valid creation order; keys: (n-1) x 4 int64.
 * Returns 0 or -1 on an invalid row, -3 on allocation failure.
 */
int oracle_merge_keys(const double *rows, int64_t n, int64_t *keys)
{
    const int64_t m = n - 1;
    if (m <= 0) return 0;
    int64_t *lo = malloc(sizeof(int64_t) * (size_t)(2 * n - 1));
    int64_t *sz = malloc(sizeof(int64_t) * (size_t)(2 * n - 1));
    if (!lo || !sz) {
        free(lo); free(sz);
        return -3;
    }
    for (int64_t i = 0; i < n; ++i) {
        lo[i] = i;
        sz[i] = 1;
    }
    int rc = 0;
    for (int64_t r = 0; r < m; ++r) {
        int64_t a = (int64_t)rows[4 * r], b = (int64_t)rows[4 * r + 1];
        if (a < 0 || b < 0 || a >= n + r || b >= n + r) {
            rc = -1;
            break;
        }
        int swap = lo[a] > lo[b] || (lo[a] == lo[b] && sz[a] > sz[b]);
        int64_t x = swap ? b : a, y = swap ? a : b;
        keys[4 * r] = lo[x];
        keys[4 * r + 1] = sz[x];
        keys[4 * r + 2] = lo[y];
        keys[4 * r + 3] = sz[y];
        lo[n + r] = lo[x];
        sz[n + r] = sz[x] + sz[y];
    }
    free(lo); free(sz);
    return rc;
}
