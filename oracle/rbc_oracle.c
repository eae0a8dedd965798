/*
 * rbc_oracle.c -- CPU FP64 oracle for the Random Ball Cover (RBC) and its
 * brute-force primitive BF(Q, X).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU library is checked against.  It shares no code with the HIP path, and
 * only tests/, the smoke entry point and the CPU-baseline leg of the bench may
 * load it.  The product path never calls it.
 *
 * Everything here is written to be checked against the paper by eye:
 *   - distances are computed in double precision from the float32 inputs
 *     (which convert exactly), by direct differences, never by the
 *     ||q||^2 + ||x||^2 - 2 q.x expansion;
 *   - ranking is lexicographic on (distance, index): the lower database id
 *     (or the lower representative position) wins a tie;
 *   - the RBC build and both search algorithms follow the paper's steps in its
 *     order: build = one BF call (Sec. 4), one-shot = BF(q,R) then BF(q,X[L_r])
 *     (Sec. 5.1), exact = BF(q,R) keeping all distances, the two pruning rules,
 *     then BF over the union of the surviving lists (Sec. 5.2).
 *
 * Readings of the paper this oracle takes (each is also listed in the design
 * notes of the repository):
 *   R1  representatives are a given set of distinct database ids, sorted
 *       ascending; "position" below is the position in that sorted list.
 *   R2  every tie is broken by (distance, index) order.
 *   R3  both pruning rules prune only on a strict inequality.  Printed as
 *       "rho(q,r) >= gamma + psi_r", rule (1) would let a representative that
 *       owns only itself (psi_r = 0) prune its own list even when it is the
 *       nearest point; the strict form keeps it.  The literal form is still
 *       available (strict = 0) so that a test can show the difference.
 *   R4  k-NN form of the rules (the paper calls the extension straightforward
 *       and does not state it): with gamma_1 <= ... <= gamma_k the k smallest
 *       representative distances (gamma_k = +inf when k > n_r),
 *         rule (1): prune r if rho(q,r) - psi_r > gamma_k,
 *         rule (2): prune r if rho(q,r) > 2 gamma_k + gamma_1,
 *       which is 3 gamma for k = 1 (Lemma 1).  Proof of (2): any point x with
 *       rho(q,x) <= gamma_k owned by r* has rho(x,r*) <= rho(x,r_1)
 *       <= gamma_k + gamma_1, hence rho(q,r*) <= 2 gamma_k + gamma_1.
 *   R5  one-shot lists hold the s nearest database points to r in (distance,
 *       index) order, r itself included; psi_r is the s-th distance.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_L2 0
#define ORC_L1 1

/* The metric rho (Sec. 4 notation; the l1 form is the one the paper writes
 * out when it defines the expansion rate in Sec. 6). */
static double rho(const float* a, const float* b, int d, int metric)
{
    double s = 0.0;
    int i;
    if (metric == ORC_L1) {
        for (i = 0; i < d; ++i) s += fabs((double)a[i] - (double)b[i]);
        return s;
    }
    for (i = 0; i < d; ++i) {
        double t = (double)a[i] - (double)b[i];
        s += t * t;
    }
    return sqrt(s);
}

/* (distance, index) lexicographic order. */
static int before(double da, int64_t ia, double db, int64_t ib)
{
    return da < db || (da == db && ia < ib);
}

typedef struct {
    double dist;
    int64_t id;
} orc_pair;

static int pair_cmp(const void* a, const void* b)
{
    const orc_pair* x = (const orc_pair*)a;
    const orc_pair* y = (const orc_pair*)b;
    if (before(x->dist, x->id, y->dist, y->id)) return -1;
    if (before(y->dist, y->id, x->dist, x->id)) return 1;
    return 0;
}

/*
 * The brute-force primitive BF(q, X[L]) of Sec. 3: compute rho(q, x) for every
 * listed x, compare, and return the k closest in (distance, index) order.
 * L == NULL means the whole database.  "index" is the database id, or the
 * position in L when by_position is set (used for BF(x, R), where ties go to
 * the lower representative position).  Unfilled slots get id -1, dist +inf.
 */
static void bf_one(const float* q, const float* X, int d, int metric,
                   const int64_t* L, int64_t nL, int k, int by_position,
                   int64_t* out_id, double* out_dist)
{
    int64_t j;
    int i;
    if (k <= 64) {
        /* insertion into a sorted list of length <= k */
        int len = 0;
        for (j = 0; j < nL; ++j) {
            int64_t row = L ? L[j] : j;
            int64_t id = by_position ? j : row;
            double dj = rho(q, X + row * (int64_t)d, d, metric);
            int pos;
            if (len == k && !before(dj, id, out_dist[k - 1], out_id[k - 1])) continue;
            pos = (len < k) ? len : k - 1;
            while (pos > 0 && before(dj, id, out_dist[pos - 1], out_id[pos - 1])) {
                out_dist[pos] = out_dist[pos - 1];
                out_id[pos] = out_id[pos - 1];
                --pos;
            }
            out_dist[pos] = dj;
            out_id[pos] = id;
            if (len < k) ++len;
        }
        for (i = len; i < k; ++i) {
            out_id[i] = -1;
            out_dist[i] = INFINITY;
        }
    } else {
        /* large k: compute every pair and sort them (library sort as a step) */
        orc_pair* all = (orc_pair*)malloc((size_t)(nL > 0 ? nL : 1) * sizeof(orc_pair));
        for (j = 0; j < nL; ++j) {
            int64_t row = L ? L[j] : j;
            all[j].dist = rho(q, X + row * (int64_t)d, d, metric);
            all[j].id = by_position ? j : row;
        }
        qsort(all, (size_t)nL, sizeof(orc_pair), pair_cmp);
        for (i = 0; i < k; ++i) {
            if (i < nL) {
                out_id[i] = all[i].id;
                out_dist[i] = all[i].dist;
            } else {
                out_id[i] = -1;
                out_dist[i] = INFINITY;
            }
        }
        free(all);
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* rho(a_i, b_i) for paired rows: used by tests for metric-axiom checks. */
int orc_rho_pairs(const float* A, const float* B, int64_t m, int32_t d, int32_t metric,
                  double* out)
{
    int64_t i;
    for (i = 0; i < m; ++i) out[i] = rho(A + i * d, B + i * d, d, metric);
    return 0;
}

/*
 * BF(Q, X), Sec. 3: for each query, k nearest database points in
 * (distance, id) order.  Q is m x d, X is n x d, both row-major float32.
 */
int orc_bf_knn(const float* Q, int64_t m, const float* X, int64_t n, int32_t d,
               int32_t metric, int32_t k, int64_t* out_idx, double* out_dist)
{
    int64_t i;
    if (d < 1 || k < 1 || n < 0 || m < 0) return -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (i = 0; i < m; ++i)
        bf_one(Q + i * (int64_t)d, X, d, metric, NULL, n, k, 0, out_idx + i * k,
               out_dist + i * k);
    return 0;
}

/*
 * Range search (the eps-range form of the problem Sec. 5 mentions beside
 * k-NN): for every query q, all database points x with rho(q, x) <= radius, in
 * (distance, index) order.  Called twice: with out_idx NULL it writes the
 * per-query counts to off[0 .. m) (the caller turns them into offsets); then
 * with off[i] .. off[i+1] the output ranges it fills them.
 */
int orc_range_bf(const float* Q, int64_t m, const float* X, int64_t n, int32_t d,
                 int32_t metric, double radius, int64_t* off, int64_t* out_idx,
                 double* out_dist)
{
    int64_t i;
    if (d < 1 || n < 0 || m < 0 || !(radius >= 0.0)) return -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (i = 0; i < m; ++i) {
        const float* q = Q + i * (int64_t)d;
        int64_t j, c = 0;
        if (!out_idx) {
            for (j = 0; j < n; ++j)
                if (rho(q, X + j * (int64_t)d, d, metric) <= radius) ++c;
            off[i] = c;
            continue;
        }
        {
            int64_t base = off[i], cnt = off[i + 1] - off[i], a, b;
            for (j = 0; j < n; ++j) {
                double r = rho(q, X + j * (int64_t)d, d, metric);
                if (r <= radius) {
                    out_idx[base + c] = j;
                    out_dist[base + c] = r;
                    ++c;
                }
            }
            /* insertion sort of the (short) result list by (distance, index) */
            for (a = 1; a < cnt; ++a) {
                double dv = out_dist[base + a];
                int64_t iv = out_idx[base + a];
                b = a - 1;
                while (b >= 0 && before(dv, iv, out_dist[base + b], out_idx[base + b])) {
                    out_dist[base + b + 1] = out_dist[base + b];
                    out_idx[base + b + 1] = out_idx[base + b];
                    --b;
                }
                out_dist[base + b + 1] = dv;
                out_idx[base + b + 1] = iv;
            }
        }
    }
    return 0;
}

/* Number of database points strictly closer to q than the given distance: the
 * rank error measure of the one-shot experiments (Sec. 7). */
int orc_rank(const float* Q, int64_t m, const float* X, int64_t n, int32_t d,
             int32_t metric, const double* ret_dist, int64_t* out_rank)
{
    int64_t i;
#pragma omp parallel for schedule(dynamic, 4)
    for (i = 0; i < m; ++i) {
        int64_t j, c = 0;
        for (j = 0; j < n; ++j)
            if (rho(Q + i * (int64_t)d, X + j * (int64_t)d, d, metric) < ret_dist[i]) ++c;
        out_rank[i] = c;
    }
    return 0;
}

/*
 * Exact-mode build (Sec. 4 and Sec. 5.2): BF(X, R) with k = 1 gives every
 * point its owner (nearest representative, ties to the lower position); L_r is
 * the set of points r owns (listed by ascending id); psi_r = max over L_r of
 * rho(x, r).
 *   owner[n]       representative position of each point
 *   psi[n_r]       radius of each list (0 for a list holding only r)
 *   list_off[n_r+1], list_ids[n]   the lists, concatenated (CSR form)
 */
int orc_rbc_build_exact(const float* X, int64_t n, int32_t d, int32_t metric,
                        const int64_t* rep_idx, int64_t n_r, int32_t* owner,
                        double* psi, int64_t* list_off, int64_t* list_ids)
{
    int64_t i, r;
    float* R;
    int64_t* fill;
    double* own_dist;
    if (n < 1 || n_r < 1 || n_r > n || d < 1) return -1;
    R = (float*)malloc((size_t)n_r * d * sizeof(float));
    own_dist = (double*)malloc((size_t)n * sizeof(double));
    for (r = 0; r < n_r; ++r) memcpy(R + r * d, X + rep_idx[r] * d, (size_t)d * sizeof(float));

#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        int64_t pos;
        double dist;
        bf_one(X + i * (int64_t)d, R, d, metric, NULL, n_r, 1, 1, &pos, &dist);
        owner[i] = (int32_t)pos;
        own_dist[i] = dist;
    }

    for (r = 0; r < n_r; ++r) psi[r] = 0.0;
    memset(list_off, 0, (size_t)(n_r + 1) * sizeof(int64_t));
    for (i = 0; i < n; ++i) {
        list_off[owner[i] + 1] += 1;
        if (own_dist[i] > psi[owner[i]]) psi[owner[i]] = own_dist[i];
    }
    for (r = 0; r < n_r; ++r) list_off[r + 1] += list_off[r];
    fill = (int64_t*)malloc((size_t)n_r * sizeof(int64_t));
    for (r = 0; r < n_r; ++r) fill[r] = list_off[r];
    for (i = 0; i < n; ++i) list_ids[fill[owner[i]]++] = i;
    free(fill);
    free(own_dist);
    free(R);
    return 0;
}

/*
 * Exact search (Sec. 5.2), k-NN form (reading R4):
 *   1. BF(q, R) keeping every distance; gamma_1, gamma_k.
 *   2. prune r by rule (1) (eq. ineq:prune) or rule (2) (eq. ineq:prune2).
 *   3. BF(q, X[L_1 u ... u L_t]) over the surviving lists.
 * strict = 1: prune only on strict inequalities (reading R3).
 * strict = 0: rule (1) as printed, rho(q,r) >= gamma_k + psi_r.
 * Outputs per query: k (id, distance) pairs in (distance, id) order; the number
 * of candidate points scanned; the number of lists kept; optionally the m x n_r
 * keep mask.
 */
/*
 * The approximate variant the paper mentions beside Sec. 5 (prune harder
 * than the exact rules allow): both rules compare against their bounds
 * divided by (1 + eps), i.e. rule 1 prunes r when rho(q,r) - psi_r >
 * gamma_k / (1 + eps) and rule 2 when rho(q,r) > (2 gamma_k + gamma_1) /
 * (1 + eps).  The result is BF(q, X[union of the kept lists]); eps = 0 is the
 * exact search above.
 */
int orc_rbc_search_approx(const float* Q, int64_t m, const float* X, int64_t n, int32_t d,
                          int32_t metric, const int64_t* rep_idx, int64_t n_r,
                          const double* psi, const int64_t* list_off,
                          const int64_t* list_ids, int32_t k, int32_t strict, double eps,
                          int64_t* out_idx, double* out_dist, int64_t* out_ncand,
                          int32_t* out_nkept, uint8_t* out_kept);

int orc_rbc_search_exact(const float* Q, int64_t m, const float* X, int64_t n, int32_t d,
                         int32_t metric, const int64_t* rep_idx, int64_t n_r,
                         const double* psi, const int64_t* list_off,
                         const int64_t* list_ids, int32_t k, int32_t strict,
                         int64_t* out_idx, double* out_dist, int64_t* out_ncand,
                         int32_t* out_nkept, uint8_t* out_kept)
{
    return orc_rbc_search_approx(Q, m, X, n, d, metric, rep_idx, n_r, psi, list_off, list_ids,
                                 k, strict, 0.0, out_idx, out_dist, out_ncand, out_nkept,
                                 out_kept);
}

int orc_rbc_search_approx(const float* Q, int64_t m, const float* X, int64_t n, int32_t d,
                          int32_t metric, const int64_t* rep_idx, int64_t n_r,
                          const double* psi, const int64_t* list_off,
                          const int64_t* list_ids, int32_t k, int32_t strict, double eps,
                          int64_t* out_idx, double* out_dist, int64_t* out_ncand,
                          int32_t* out_nkept, uint8_t* out_kept)
{
    int64_t i;
    const double shrink = 1.0 / (1.0 + eps);
    if (k < 1 || k > n || d < 1 || !(eps >= 0.0)) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (i = 0; i < m; ++i) {
        const float* q = Q + i * (int64_t)d;
        double* dr = (double*)malloc((size_t)n_r * sizeof(double));
        double* srt = (double*)malloc((size_t)n_r * sizeof(double));
        int64_t* cand;
        int64_t r, ncand = 0, j;
        int32_t nkept = 0;
        double g1, gk;

        /* step 1: BF(q, R), all distances retained */
        for (r = 0; r < n_r; ++r) {
            dr[r] = rho(q, X + rep_idx[r] * (int64_t)d, d, metric);
            srt[r] = dr[r];
        }
        /* gamma_1 = min, gamma_k = k-th smallest (+inf if k > n_r) */
        {
            int64_t a, b;
            int64_t kk = (k < n_r) ? k : n_r;
            for (a = 0; a < kk; ++a) /* partial selection sort of the k smallest */
                for (b = a + 1; b < n_r; ++b)
                    if (srt[b] < srt[a]) {
                        double t = srt[a];
                        srt[a] = srt[b];
                        srt[b] = t;
                    }
            g1 = srt[0];
            gk = (k <= n_r) ? srt[k - 1] : INFINITY;
        }

        /* step 2: pruning rules (1) and (2) */
        for (r = 0; r < n_r; ++r) {
            int prune1 = strict ? (dr[r] - psi[r] > gk * shrink) : (dr[r] >= gk * shrink + psi[r]);
            int prune2 = dr[r] > (2.0 * gk + g1) * shrink;
            int keep = !(prune1 || prune2);
            if (out_kept) out_kept[i * n_r + r] = (uint8_t)keep;
            if (keep) {
                ++nkept;
                ncand += list_off[r + 1] - list_off[r];
            }
        }

        /* step 3: BF(q, X[union of surviving lists]) */
        cand = (int64_t*)malloc((size_t)(ncand > 0 ? ncand : 1) * sizeof(int64_t));
        j = 0;
        for (r = 0; r < n_r; ++r) {
            int prune1 = strict ? (dr[r] - psi[r] > gk * shrink) : (dr[r] >= gk * shrink + psi[r]);
            int prune2 = dr[r] > (2.0 * gk + g1) * shrink;
            if (!(prune1 || prune2)) {
                int64_t t;
                for (t = list_off[r]; t < list_off[r + 1]; ++t) cand[j++] = list_ids[t];
            }
        }
        bf_one(q, X, d, metric, cand, ncand, k, 0, out_idx + i * k, out_dist + i * k);
        if (out_ncand) out_ncand[i] = ncand;
        if (out_nkept) out_nkept[i] = nkept;
        free(cand);
        free(srt);
        free(dr);
    }
    return 0;
}

/*
 * One-shot build (Sec. 4 and Sec. 5.1, reading R5): BF(R, X) with k = s, i.e.
 * L_r = the s nearest database points to r in (distance, id) order, and
 * psi_r = the s-th of those distances.  lists is n_r x s (ids), row r for the
 * r-th representative of rep_idx (any subset of representatives may be
 * passed; each list depends only on its own representative).
 */
int orc_rbc_build_oneshot(const float* X, int64_t n, int32_t d, int32_t metric,
                          const int64_t* rep_idx, int64_t n_r, int64_t s,
                          int64_t* lists, double* psi)
{
    int64_t r;
    if (s < 1 || s > n || d < 1) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (r = 0; r < n_r; ++r) {
        double* dist = (double*)malloc((size_t)s * sizeof(double));
        bf_one(X + rep_idx[r] * (int64_t)d, X, d, metric, NULL, n, (int)s, 0,
               lists + r * s, dist);
        psi[r] = dist[s - 1];
        free(dist);
    }
    return 0;
}

/*
 * One-shot search (Sec. 5.1): r = BF(q, R) (nearest representative, ties to
 * the lower position), then BF(q, X[L_r]).  out_rep receives r's position.
 */
int orc_rbc_search_oneshot(const float* Q, int64_t m, const float* X, int64_t n, int32_t d,
                           int32_t metric, const int64_t* rep_idx, int64_t n_r, int64_t s,
                           const int64_t* lists, int32_t k, int64_t* out_idx,
                           double* out_dist, int64_t* out_rep)
{
    int64_t i;
    if (k < 1 || k > s || d < 1) return -1;
    (void)n;
#pragma omp parallel for schedule(dynamic, 4)
    for (i = 0; i < m; ++i) {
        const float* q = Q + i * (int64_t)d;
        int64_t best = -1, r;
        double bd = INFINITY;
        for (r = 0; r < n_r; ++r) {
            double dr = rho(q, X + rep_idx[r] * (int64_t)d, d, metric);
            if (best < 0 || dr < bd) { /* ascending r: a tie keeps the lower position */
                bd = dr;
                best = r;
            }
        }
        out_rep[i] = best;
        bf_one(q, X, d, metric, lists + best * s, s, k, 0, out_idx + i * k, out_dist + i * k);
    }
    return 0;
}
