/*
 * mdfs_oracle.c -- plain, slow FP64 reference of the MDFS k-tuple information-gain sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this file:
 * only the tests, the smoke check and the CPU-baseline leg of the benchmark use it.  It shares
 * no code, header, table or constant generator with the HIP implementation.
 *
 * What it computes (paper: "MDFS - MultiDimensional Feature Selection", Piliszek et al.):
 *   * randomised rank-based discretisation (section "Algorithm and implementation", the
 *     paragraph on range and shares), repeated over several random discretisations;
 *   * per-class voxel counts of every k-tuple (same section, the counters N^d);
 *   * pseudocounted class probabilities (the p^d and beta^d equations of that section);
 *   * conditional entropy, read as the voxel-weighted sum  H(y|X) = sum_v (n_v/N) h(p_v)
 *     (the printed entropy equation omits the voxel weight; see the readings list);
 *   * IG^k_max(y;x_i) = N max_m (H(y|x_m..) - H(y|x_i,x_m..))  (equation IGmax, section
 *     "Theory"), maximised over tuples and discretisations, with the tuple and the
 *     discretisation where the maximum is attained.
 *
 * Readings of passages the paper leaves open (all listed in the design notes):
 *   R1 RNG: counter-based SplitMix64 (Steele, Lea & Flood 2014) keyed by (seed, disc, var, j).
 *   R2 shares s_j = (1-range) + 2*range*u_j; cut t_j = floor(N*cum_j/S) for j=1..c-1, clamped to
 *      [1, N-1], forced strictly increasing and <= N-(c-j); thresholds v_j = sorted(x)[t_j];
 *      code = #{j : x >= v_j}  (a value equal to a threshold goes to the upper class).
 *   R3 pseudocount: the numerator of the class-probability equation prints beta^k; read beta^d.
 *   R4 entropy weight: H(y|X) = sum_v (n_v/N) h(p_v), natural logarithm; so N*H = F = sum n_v h.
 *   R5 xi = 0 uses 0 ln 0 = 0 (test-only).
 *   R6 ties: candidates with IG >= max - tau, tau = 1e-9*max(1,|max|), are tied; the smallest
 *      discretisation index wins, then the lexicographically smallest partner tuple.
 *   R7 voxel terms of F are summed in ascending order, so a table and any permutation of its
 *      axes give bit-identical F.
 *
 * All floating-point arithmetic is IEEE binary64 with no contraction (built -ffp-contract=off,
 * no fast-math).  Arrays are variable-major: data[var*n_obj + obj], codes[(r*n_var+var)*n_obj+obj].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OK = 0, E_ARG = -1, E_Y = -2, E_K = -3, E_DIV = -4, E_NAN = -5, E_NOMEM = -6 };

#define MAXK 5

/* ---------------------------------------------------------------- R1: SplitMix64 */
static uint64_t sm_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
static const uint64_t SM_GAMMA = 0x9e3779b97f4a7c15ULL;

/* The sequential generator, exported only so the tests can check it against the published
 * first outputs for state 0. */
uint64_t mdfs_oracle_splitmix64_next(uint64_t *state)
{
    *state += SM_GAMMA;
    return sm_mix(*state);
}

/* Counter-based draw for (seed, discretisation, variable, share index): each key component is
 * absorbed by one SplitMix64 step whose state is the previous output plus (component+1)*gamma. */
uint64_t mdfs_oracle_draw(uint64_t seed, int64_t disc, int64_t var, int64_t j)
{
    uint64_t h = sm_mix(seed + SM_GAMMA);
    h = sm_mix(h + (uint64_t)(disc + 1) * SM_GAMMA);
    h = sm_mix(h + (uint64_t)(var + 1) * SM_GAMMA);
    h = sm_mix(h + (uint64_t)(j + 1) * SM_GAMMA);
    return h;
}

/* ---------------------------------------------------------------- R2: cut positions */
/* c shares drawn from U(1-range, 1+range); c-1 cut positions in the sorted variable. */
int mdfs_oracle_cuts(int64_t n_obj, int c, double range, uint64_t seed, int64_t disc, int64_t var,
                     int64_t *t)
{
    if (c < 2 || n_obj < c || !(range >= 0.0 && range <= 1.0)) return E_ARG;
    double s[16];
    if (c > 16) return E_DIV;
    for (int j = 0; j < c; ++j) {
        double u = (double)(mdfs_oracle_draw(seed, disc, var, j) >> 11) * (1.0 / 9007199254740992.0);
        s[j] = (1.0 - range) + (2.0 * range) * u;
    }
    double S = 0.0;
    for (int j = 0; j < c; ++j) S = S + s[j];
    double cum = 0.0;
    int64_t prev = 0;
    for (int j = 1; j < c; ++j) {
        cum = cum + s[j - 1];
        double q = ((double)n_obj * cum) / S;
        int64_t tj = (int64_t)floor(q);
        if (tj < 1) tj = 1;
        if (tj > n_obj - 1) tj = n_obj - 1;
        if (j > 1 && tj < prev + 1) tj = prev + 1;
        if (tj > n_obj - (c - j)) tj = n_obj - (c - j);
        t[j - 1] = tj;
        prev = tj;
    }
    return OK;
}

static int cmp_float(const void *a, const void *b)
{
    float x = *(const float *)a, y = *(const float *)b;
    return (x > y) - (x < y);
}

/* Discretise every variable under discretisations disc_offset .. disc_offset+n_disc-1.
 * codes: [n_disc][n_var][n_obj] uint8, each in [0, divisions]. */
int mdfs_oracle_discretize(const float *data, int64_t n_obj, int64_t n_var, int divisions,
                           int64_t n_disc, int64_t disc_offset, double range, uint64_t seed,
                           uint8_t *codes)
{
    int c = divisions + 1;
    if (!data || !codes || n_obj <= 0 || n_var <= 0 || n_disc <= 0 || disc_offset < 0) return E_ARG;
    if (divisions < 1 || c > 16) return E_DIV;
    if (n_obj < c) return E_ARG;
    for (int64_t i = 0; i < n_var * n_obj; ++i)
        if (isnan(data[i])) return E_NAN;
    float *sorted = (float *)malloc(sizeof(float) * (size_t)n_obj);
    if (!sorted) return E_NOMEM;
    for (int64_t v = 0; v < n_var; ++v) {
        const float *x = data + v * n_obj;
        memcpy(sorted, x, sizeof(float) * (size_t)n_obj);
        qsort(sorted, (size_t)n_obj, sizeof(float), cmp_float);
        for (int64_t r = 0; r < n_disc; ++r) {
            int64_t t[16];
            float thr[16];
            int rc = mdfs_oracle_cuts(n_obj, c, range, seed, disc_offset + r, v, t);
            if (rc) { free(sorted); return rc; }
            for (int j = 0; j < c - 1; ++j) thr[j] = sorted[t[j]];
            uint8_t *out = codes + (r * n_var + v) * n_obj;
            for (int64_t n = 0; n < n_obj; ++n) {
                int code = 0;
                for (int j = 0; j < c - 1; ++j)
                    if (x[n] >= thr[j]) code++;
                out[n] = (uint8_t)code;
            }
        }
    }
    free(sorted);
    return OK;
}

/* ---------------------------------------------------------------- counts */
/* Per-class voxel counts of the k-tuple `vars` (any order) under one discretisation.
 * table: [2][c^k], class-major; cell index is mixed radix with vars[0] most significant. */
int mdfs_oracle_table(const uint8_t *codes_r, const uint8_t *y, int64_t n_obj, int c, int k,
                      const int64_t *vars, int64_t *table)
{
    int64_t ncell = 1;
    for (int m = 0; m < k; ++m) ncell *= c;
    memset(table, 0, sizeof(int64_t) * (size_t)(2 * ncell));
    for (int64_t n = 0; n < n_obj; ++n) {
        int64_t cell = 0;
        for (int m = 0; m < k; ++m) cell = cell * c + codes_r[vars[m] * n_obj + n];
        table[(int64_t)y[n] * ncell + cell] += 1;
    }
    return OK;
}

/* Class sizes and beta^d = xi * N^d / min(N^0, N^1). */
int mdfs_oracle_betas(const uint8_t *y, int64_t n_obj, double xi, double *beta0, double *beta1)
{
    int64_t n1 = 0;
    for (int64_t n = 0; n < n_obj; ++n) {
        if (y[n] > 1) return E_Y;
        n1 += y[n];
    }
    int64_t n0 = n_obj - n1;
    if (n0 == 0 || n1 == 0) return E_Y;
    double m = (double)(n0 < n1 ? n0 : n1);
    *beta0 = xi * (double)n0 / m;
    *beta1 = xi * (double)n1 / m;
    return OK;
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* F(table) = sum_v n_v * h(p_v),  h(p) = -sum_d p^d ln p^d,
 * p^d_v = (n^d_v + beta^d) / (n^0_v + beta^0 + n^1_v + beta^1).  Terms summed ascending (R7). */
double mdfs_oracle_F(const int64_t *table, int64_t ncell, double beta0, double beta1)
{
    double *terms = (double *)malloc(sizeof(double) * (size_t)ncell);
    int64_t nt = 0;
    for (int64_t v = 0; v < ncell; ++v) {
        double n0 = (double)table[v], n1 = (double)table[ncell + v];
        double nv = n0 + n1;
        if (nv == 0.0) continue; /* zero weight */
        double den = n0 + beta0 + n1 + beta1;
        double p0 = (n0 + beta0) / den, p1 = (n1 + beta1) / den;
        double h = 0.0;
        if (p0 > 0.0) h -= p0 * log(p0);
        if (p1 > 0.0) h -= p1 * log(p1);
        terms[nt++] = nv * h;
    }
    qsort(terms, (size_t)nt, sizeof(double), cmp_double);
    double F = 0.0;
    for (int64_t t = 0; t < nt; ++t) F = F + terms[t];
    free(terms);
    return F;
}

/* ---------------------------------------------------------------- R6: tie rule */
typedef struct {
    double v;
    int64_t r;
    int64_t m[MAXK];
} cand_t;
typedef struct {
    double best;
    int64_t n, cap;
    cand_t *c;
} best_t;

static double tau_of(double m) { return 1e-9 * (fabs(m) > 1.0 ? fabs(m) : 1.0); }

static int key_less(const cand_t *a, const cand_t *b, int km1)
{
    if (a->r != b->r) return a->r < b->r;
    for (int q = 0; q < km1; ++q)
        if (a->m[q] != b->m[q]) return a->m[q] < b->m[q];
    return 0;
}

static void best_init(best_t *b)
{
    b->best = -INFINITY;
    b->n = 0;
    b->cap = 0;
    b->c = NULL;
}

static int best_offer(best_t *b, const cand_t *x)
{
    if (x->v > b->best) {
        b->best = x->v;
        double lo = b->best - tau_of(b->best);
        int64_t w = 0;
        for (int64_t q = 0; q < b->n; ++q)
            if (b->c[q].v >= lo) b->c[w++] = b->c[q];
        b->n = w;
    }
    if (x->v >= b->best - tau_of(b->best)) {
        if (b->n == b->cap) {
            int64_t nc = b->cap ? 2 * b->cap : 4;
            cand_t *p = (cand_t *)realloc(b->c, sizeof(cand_t) * (size_t)nc);
            if (!p) return E_NOMEM;
            b->c = p;
            b->cap = nc;
        }
        b->c[b->n++] = *x;
    }
    return OK;
}

/* Winner among the surviving candidates: smallest discretisation, then lexicographic tuple. */
static const cand_t *best_pick(const best_t *b, int km1)
{
    const cand_t *w = NULL;
    double lo = b->best - tau_of(b->best);
    for (int64_t q = 0; q < b->n; ++q) {
        if (b->c[q].v < lo) continue;
        if (!w || key_less(&b->c[q], w, km1)) w = &b->c[q];
    }
    return w;
}

/* ---------------------------------------------------------------- subsets */
/* Advance a sorted k-subset of {0..n-1} to the next in lexicographic order; 0 when done. */
static int next_subset(int64_t *s, int k, int64_t n)
{
    int q = k - 1;
    while (q >= 0 && s[q] == n - k + q) --q;
    if (q < 0) return 0;
    s[q]++;
    for (int t = q + 1; t < k; ++t) s[t] = s[t - 1] + 1;
    return 1;
}

static int check_common(const float *data, const uint8_t *y, int64_t n_obj, int64_t n_var, int k,
                        int divisions, int64_t n_disc, double xi)
{
    if (!data || !y || n_obj <= 0 || n_var <= 0 || n_disc <= 0) return E_ARG;
    if (k < 1 || k > MAXK || k > n_var) return E_K;
    if (divisions < 1 || divisions > 15) return E_DIV;
    if (n_obj < divisions + 1) return E_ARG;
    if (!(xi >= 0.0)) return E_ARG;
    return OK;
}

/* IG of one member of one tuple: F(T \ {member}) - F(T) under discretisation codes_r.
 * vars: the k variables of T (sorted or not), member: position of x_i within vars. */
double mdfs_oracle_ig_member(const uint8_t *codes_r, const uint8_t *y, int64_t n_obj, int c, int k,
                             const int64_t *vars, int member, double beta0, double beta1)
{
    int64_t ncell = 1;
    for (int m = 0; m < k; ++m) ncell *= c;
    int64_t *tab = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * ncell));
    int64_t rest[MAXK];
    int q = 0;
    for (int m = 0; m < k; ++m)
        if (m != member) rest[q++] = vars[m];
    mdfs_oracle_table(codes_r, y, n_obj, c, k, vars, tab);
    double FT = mdfs_oracle_F(tab, ncell, beta0, beta1);
    mdfs_oracle_table(codes_r, y, n_obj, c, k - 1, rest, tab);
    double FM = mdfs_oracle_F(tab, ncell / c, beta0, beta1);
    free(tab);
    return FM - FT;
}

/* IG^k_max for the listed target variables, straight from the IGmax equation: for each target
 * x_i, every discretisation r and every (k-1)-subset M of the other variables (lexicographic),
 * IG(i|M) = F(M) - F(M u {i}), each F counted from its own table.  Targets are independent, so
 * they are shared among n_threads OpenMP threads.
 * Outputs: ig[n_targets], argmax[n_targets][k-1] (ascending variable indices; -1 for k=1),
 * argdisc[n_targets] (absolute discretisation index = disc_offset + r). */
int mdfs_oracle_max_ig(const float *data, const uint8_t *y, int64_t n_obj, int64_t n_var, int k,
                       int divisions, int64_t n_disc, int64_t disc_offset, double range, double xi,
                       uint64_t seed, const int64_t *targets, int64_t n_targets, double *ig,
                       int64_t *argmax, int64_t *argdisc, int n_threads)
{
    int rc = check_common(data, y, n_obj, n_var, k, divisions, n_disc, xi);
    if (rc) return rc;
    double b0, b1;
    if ((rc = mdfs_oracle_betas(y, n_obj, xi, &b0, &b1))) return rc;
    int c = divisions + 1;
    uint8_t *codes = (uint8_t *)malloc((size_t)(n_disc * n_var * n_obj));
    if (!codes) return E_NOMEM;
    rc = mdfs_oracle_discretize(data, n_obj, n_var, divisions, n_disc, disc_offset, range, seed, codes);
    if (rc) { free(codes); return rc; }
    int km1 = k - 1;
    int fail = 0;
#ifdef _OPENMP
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
#endif
    for (int64_t ti = 0; ti < n_targets; ++ti) {
        int64_t i = targets[ti];
        if (i < 0 || i >= n_var) { fail = 1; continue; }
        best_t b;
        best_init(&b);
        for (int64_t r = 0; r < n_disc; ++r) {
            const uint8_t *cr = codes + r * n_var * n_obj;
            int64_t others[MAXK], s[MAXK];
            for (int q = 0; q < km1; ++q) s[q] = q;
            int more = (km1 == 0) || (n_var - 1 >= km1);
            while (more) {
                /* map the subset of {0..n_var-2} to variables other than i */
                int64_t vars[MAXK];
                for (int q = 0; q < km1; ++q) others[q] = s[q] < i ? s[q] : s[q] + 1;
                int pos = 0, member = 0;
                for (int q = 0; q < km1; ++q) {
                    if (others[q] > i && pos == q) { vars[pos++] = i; member = q; }
                    vars[pos++] = others[q];
                }
                if (pos == km1) { member = km1; vars[pos++] = i; }
                cand_t x;
                x.v = mdfs_oracle_ig_member(cr, y, n_obj, c, k, vars, member, b0, b1);
                x.r = disc_offset + r;
                for (int q = 0; q < km1; ++q) x.m[q] = others[q];
                if (best_offer(&b, &x)) fail = 1;
                more = km1 > 0 && next_subset(s, km1, n_var - 1);
            }
        }
        const cand_t *w = best_pick(&b, km1);
        ig[ti] = b.best;
        argdisc[ti] = w ? w->r : -1;
        for (int q = 0; q < (km1 > 0 ? km1 : 1); ++q) argmax[ti * (km1 > 0 ? km1 : 1) + q] = (w && km1 > 0) ? w->m[q] : -1;
        free(b.c);
    }
    free(codes);
    return fail ? E_NOMEM : OK;
}

/* The same quantity for all variables, organised as the sweep the paper describes: every
 * k-subset T (lexicographic) is counted once, F(T) is evaluated, and each member i is credited
 * IG(i | T\{i}) = F(marginal of T over i) - F(T); the marginal is the exact (k-1)-table of
 * T\{i}.  Discretisations are shared among n_threads threads, each keeping its own candidate
 * sets; the sets are merged with the same tie rule, so the result does not depend on n_threads. */
int mdfs_oracle_max_ig_all(const float *data, const uint8_t *y, int64_t n_obj, int64_t n_var, int k,
                           int divisions, int64_t n_disc, int64_t disc_offset, double range, double xi,
                           uint64_t seed, double *ig, int64_t *argmax, int64_t *argdisc, int n_threads)
{
    int rc = check_common(data, y, n_obj, n_var, k, divisions, n_disc, xi);
    if (rc) return rc;
    double b0, b1;
    if ((rc = mdfs_oracle_betas(y, n_obj, xi, &b0, &b1))) return rc;
    int c = divisions + 1;
    int km1 = k - 1;
    uint8_t *codes = (uint8_t *)malloc((size_t)(n_disc * n_var * n_obj));
    if (!codes) return E_NOMEM;
    rc = mdfs_oracle_discretize(data, n_obj, n_var, divisions, n_disc, disc_offset, range, seed, codes);
    if (rc) { free(codes); return rc; }
    if (n_threads < 1) n_threads = 1;
    if (n_threads > n_disc) n_threads = (int)n_disc;
    best_t *bests = (best_t *)malloc(sizeof(best_t) * (size_t)(n_threads * n_var));
    for (int64_t q = 0; q < n_threads * n_var; ++q) best_init(&bests[q]);
    int64_t ncell = 1;
    for (int m = 0; m < k; ++m) ncell *= c;
    int fail = 0;
#ifdef _OPENMP
#pragma omp parallel num_threads(n_threads)
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        best_t *mine = bests + (int64_t)tid * n_var;
        int64_t *tab = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * ncell));
        int64_t *sub = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * ncell));
        for (int64_t r = tid; r < n_disc; r += n_threads) {
            const uint8_t *cr = codes + r * n_var * n_obj;
            int64_t T[MAXK];
            for (int q = 0; q < k; ++q) T[q] = q;
            do {
                mdfs_oracle_table(cr, y, n_obj, c, k, T, tab);
                double FT = mdfs_oracle_F(tab, ncell, b0, b1);
                for (int mem = 0; mem < k; ++mem) {
                    /* marginalise the table over axis `mem` */
                    int64_t sc = ncell / c;
                    memset(sub, 0, sizeof(int64_t) * (size_t)(2 * sc));
                    for (int64_t cell = 0; cell < ncell; ++cell) {
                        int64_t digits[MAXK], rem = cell;
                        for (int q = k - 1; q >= 0; --q) { digits[q] = rem % c; rem /= c; }
                        int64_t sidx = 0;
                        for (int q = 0; q < k; ++q)
                            if (q != mem) sidx = sidx * c + digits[q];
                        sub[sidx] += tab[cell];
                        sub[sc + sidx] += tab[ncell + cell];
                    }
                    cand_t x;
                    x.v = mdfs_oracle_F(sub, sc, b0, b1) - FT;
                    x.r = disc_offset + r;
                    int q2 = 0;
                    for (int q = 0; q < k; ++q)
                        if (q != mem) x.m[q2++] = T[q];
                    if (best_offer(&mine[T[mem]], &x)) fail = 1;
                }
            } while (next_subset(T, k, n_var));
        }
        free(tab);
        free(sub);
    }
    for (int64_t v = 0; v < n_var; ++v) {
        best_t merged;
        best_init(&merged);
        for (int t = 0; t < n_threads; ++t) {
            best_t *b = &bests[(int64_t)t * n_var + v];
            for (int64_t q = 0; q < b->n; ++q)
                if (best_offer(&merged, &b->c[q])) fail = 1;
            free(b->c);
        }
        const cand_t *w = best_pick(&merged, km1);
        ig[v] = merged.best;
        argdisc[v] = w ? w->r : -1;
        for (int q = 0; q < (km1 > 0 ? km1 : 1); ++q) argmax[v * (km1 > 0 ? km1 : 1) + q] = (w && km1 > 0) ? w->m[q] : -1;
        free(merged.c);
    }
    free(bests);
    free(codes);
    return fail ? E_NOMEM : OK;
}

/* Threads OpenMP would use (1 when built without OpenMP). */
/* ComputeInterestingTuples (section "Canonical package usage"): every (variable i, partner
 * tuple m, discretisation r) with IG(i | m) >= ig_thr, IG as in max_ig_all (the table of the
 * tuple T = {i} u m, marginalised over i for the parent).  Records go out in the order r, then
 * T lexicographic, then member; at most cap are written, the return value is the number found
 * (negative on error).  var[q], partners[q][k-1], disc[q], igv[q]. */
int64_t mdfs_oracle_interesting(const float *data, const uint8_t *y, int64_t n_obj, int64_t n_var, int k,
                                int divisions, int64_t n_disc, int64_t disc_offset, double range, double xi,
                                uint64_t seed, double ig_thr, int64_t cap, int64_t *var, int64_t *partners,
                                int64_t *disc, double *igv)
{
    int rc = check_common(data, y, n_obj, n_var, k, divisions, n_disc, xi);
    if (rc) return rc;
    double b0, b1;
    if ((rc = mdfs_oracle_betas(y, n_obj, xi, &b0, &b1))) return rc;
    const int c = divisions + 1, km1 = k - 1;
    uint8_t *codes = (uint8_t *)malloc((size_t)(n_disc * n_var * n_obj));
    if (!codes) return E_NOMEM;
    rc = mdfs_oracle_discretize(data, n_obj, n_var, divisions, n_disc, disc_offset, range, seed, codes);
    if (rc) { free(codes); return rc; }
    int64_t ncell = 1;
    for (int m = 0; m < k; ++m) ncell *= c;
    int64_t *tab = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * ncell));
    int64_t *sub = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * ncell));
    int64_t found = 0;
    for (int64_t r = 0; r < n_disc; ++r) {
        const uint8_t *cr = codes + r * n_var * n_obj;
        int64_t T[MAXK];
        for (int q = 0; q < k; ++q) T[q] = q;
        do {
            mdfs_oracle_table(cr, y, n_obj, c, k, T, tab);
            const double FT = mdfs_oracle_F(tab, ncell, b0, b1);
            for (int mem = 0; mem < k; ++mem) {
                const int64_t sc = ncell / c;
                memset(sub, 0, sizeof(int64_t) * (size_t)(2 * sc));
                for (int64_t cell = 0; cell < ncell; ++cell) {
                    int64_t digits[MAXK], rem = cell;
                    for (int q = k - 1; q >= 0; --q) { digits[q] = rem % c; rem /= c; }
                    int64_t sidx = 0;
                    for (int q = 0; q < k; ++q)
                        if (q != mem) sidx = sidx * c + digits[q];
                    sub[sidx] += tab[cell];
                    sub[sc + sidx] += tab[ncell + cell];
                }
                const double g = mdfs_oracle_F(sub, sc, b0, b1) - FT;
                if (!(g >= ig_thr)) continue;
                if (found < cap) {
                    var[found] = T[mem];
                    int q2 = 0;
                    for (int q = 0; q < k; ++q)
                        if (q != mem) partners[found * km1 + q2++] = T[q];
                    disc[found] = disc_offset + r;
                    igv[found] = g;
                }
                ++found;
            }
        } while (next_subset(T, k, n_var));
    }
    free(tab);
    free(sub);
    free(codes);
    return found;
}

int mdfs_oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
