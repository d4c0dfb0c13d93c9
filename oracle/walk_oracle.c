/*
 * CPU oracle for the dynamic random-walk transition sampler.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may load this file: only the
 * test-suite, the package smoke check and the benchmark's CPU-baseline leg do.  It
 * shares no code with the GPU implementation.
 *
 * It is written to be read against FlexiWalker (arXiv 2512.00705):
 *   - transition weight and probability: w~ = w * h, p(u) = w~(v,u) / sum_t w~(v,t)
 *     (Section 2.1, Eq. prob);
 *   - Node2Vec workload weight 1/a, 1, 1/b by dist(v', u) = 0, 1, 2 (Eq. node2vec);
 *     a and b are called p and q here;
 *   - MetaPath: weight 1 when the edge label matches the schema position, else 0
 *     (Section 2.1);
 *   - Second-order PageRank (Eq. 2ndpr): with max_d = max(d(v), d(v')), weight
 *     ((1-g)/d(v) + g/d(v')) * max_d when u is a neighbour of v', ((1-g)/d(v)) * max_d
 *     otherwise; the first step has no v' and uses weight 1;
 *   - eRVS: exponential keys k_i = u_i^(1/w~_i), argmax wins, ">=" so later items win
 *     ties (Section 3.2, Algorithm 1), plus the jump of Eq. (jump) run per lane with a
 *     shared initial maximum (Section 3.2, parallel description); optionally (plan
 *     rvs_share) the lanes also take the largest threshold among them after each round
 *     in which one drew a key, their remaining skips rescaled to it (an extension: the
 *     remaining skip is exponential, so the rescaled skip is that of the new threshold);
 *   - eRJS: uniform proposal, accept when U * c' < w~ for any bound c' >= max w~
 *     (Section 3.3 and its proof);
 *   - bound max(w) * max(h) and sum estimate mean(w) * sum(h) (Section 3.3, Section 4.2
 *     helper generation, Eq. sum_estimation);
 *   - cost model: choose eRJS iff (EdgeCost_RJS / EdgeCost_RVS) * max w~ < sum w~
 *     (Section 4.1, Eq. runtime).
 *   - optional h-proportional proposals (plan.proposal = 1, not in the paper): eRJS
 *     proposes u with probability h(v,u) / sum h from a per-row alias table of the static
 *     property weights (Walker's alias method, Vose's construction) and accepts with
 *     w(u) / W for W >= every workload weight; the mass of u is then h * w / (W * sum h),
 *     proportional to w~, so the distribution is unchanged and the expected trials drop
 *     from deg * max(w) * h_MAX / S to W * sum h / S;
 *   - optional label-conditioned proposals for MetaPath (plan.proposal = 2, not in the
 *     paper; other logics take the h-proportional proposals above): a MetaPath weight is
 *     h when the edge label is the schema's, else 0, so with an alias table per (vertex,
 *     label) group of the static h one proposal from the wanted label's group is already
 *     a sample of the step: eRJS with a bound that equals every weight, one trial;
 *   - optional member board (plan.bound = 2, not in the paper) for logics whose weight is
 *     larger on N(v') than off it (Node2Vec with q > 1, second-order PageRank with g > 0):
 *     regular columns at the lower weight w_oth take every proposal (members included),
 *     a member region of area (w_mem - w_oth) * h_MAX * d(v') picks a neighbour x of v'
 *     uniformly and keeps it when x is in N(v) with probability h(v,x) / h_MAX, so each
 *     member gets the extra mass (w_mem - w_oth) * h(v,x); the return edge keeps its own
 *     column.  Per step the smaller of this board and the split/plain board is used;
 *   - optional split bound for Node2Vec (plan.bound = 1, not in the paper; any bound
 *     that dominates w~ keeps rejection sampling exact, Section 3.3): the return edge
 *     is the only one weighted 1/p, so the proposal board is deg columns of height
 *     Bn = max(1, 1/q) * h_MAX plus one extra column of height E = max(0, w~ret - Bn)
 *     that belongs to the return edge.  A trial lands in the extra column with
 *     probability E / (deg * Bn + E) and then takes the return edge; otherwise it is
 *     the usual uniform proposal against height Bn.  Each edge's total acceptance
 *     mass is min(w~, Bn) + [return] E = w~, so the distribution is unchanged; the
 *     expected trials drop from deg * B / S to (deg * Bn + E) / S.
 *
 * Canonical stream.  To compare samples one by one with a GPU run the random numbers
 * are a fixed function of (seed, walker, step, draw): Philox4x32-10 (Salmon, Moraes,
 * Dror, Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3", SC'11) with key = seed and
 * counter = (walker, step, draw, tag); tag 0 = eRJS trial, 1 = eRVS item, 3 = ITS,
 * 4 = random selection.
 * All sampling arithmetic is IEEE float32 with round-to-nearest and no contraction;
 * logarithms are evaluated in double and rounded once to float32.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC walk_oracle.c -lm
 *
 * OG_MUTANT (tests only) plants one known mistake so that the test-suite can show its
 * pins catch it: 1 swaps the Node2Vec return weight 1/p for 1/q, 2 drops the
 * conditioning of the jump key, 3 keeps the skip sum after a jump, 4 never proposes
 * the last neighbour in eRJS, 5 drops h_MAX from the eRJS bound, 6 makes the split
 * bound's extra column the full return weight instead of its excess over Bn, 7 divides
 * the second-order PageRank term g by d(v) instead of d(v'), 8 never takes an alias
 * table's alias (every slot keeps itself), 9 lets the member region keep a member without
 * its h(v, x) / h_MAX test, 10 averages the Node2Vec return values over 2 instead of their 3
 * branches in the sum estimate, 11 inverts the cost model's choice, 12 charges 8 bytes
 * instead of 16 for the row pointer pair of a step, 13 builds a label group's alias table
 * from the whole row's h maximum and ignores the group's weights (uniform within the group),
 * 14 inverts the ratio that rescales a lane's skip to a shared eRVS threshold, 15 shares the
 * threshold without rescaling the skip.
 */
#ifndef OG_MUTANT
#define OG_MUTANT 0
#endif
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ Philox4x32-10 */
/* Round function and constants as published by Salmon et al. (SC'11). */
void og_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform on the open interval (0,1): (2m+1) * 2^-24 with m the top 23 bits.
 * Every value is exact in float32 and the set is symmetric about 1/2. */
float og_uniform(uint32_t x)
{
    return (float)(2u * (x >> 9) + 1u) * 0x1p-24f;
}

static void draw(uint64_t seed, uint32_t walker, uint32_t step, uint32_t idx, uint32_t tag, uint32_t out[4])
{
    uint32_t ctr[4] = {walker, step, idx, tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    og_philox(ctr, key, out);
}

/* 8-bit property weights (Section 7, low-precision edge weights): the weight of a code
 * is h_scale * code, one float32 product rounded to nearest. */
void og_dequantize_h8(const uint8_t *code, float h_scale, int64_t n, float *h)
{
    for (int64_t k = 0; k < n; ++k) h[k] = (float)code[k] * h_scale;
}

/* Transcendentals: exact value (double libm) rounded once to float32. */
static float ln_f(float x) { return (float)log((double)x); }
static float expm1_f(float x) { return (float)expm1((double)x); }
static float log1p_f(float x) { return (float)log1p((double)x); }

/* ------------------------------------------------------------------ inputs */
typedef struct {
    int64_t nv, ne;
    const int64_t *row_ptr;
    const int32_t *col;
    const float *h;       /* NULL: unweighted (h = 1) */
    const uint8_t *label; /* NULL unless MetaPath */
    const uint32_t *alias_thr; /* per entry: keep-threshold of its alias slot (og_build_alias), or NULL */
    const int32_t *alias_idx;  /* per entry: row offset of its alias */
    int32_t h8;                /* 1: h holds dequantised 8-bit codes (og_dequantize_h8); a scanned
                                  or proposed edge then moves 1 byte of weight instead of 4 */
    /* label groups (og_build_label_alias), or NULL: nlab labels 0..nlab-1; lrow[v * nlab + l]
       is the first position of group (v, l) in grouped order, lrow[nv * nlab] = ne; per
       grouped position its row offset (lperm), keep-threshold (lthr) and alias slot within
       the group (lalias) */
    int32_t nlab;
    const int64_t *lrow;
    const int32_t *lperm;
    const uint32_t *lthr;
    const int32_t *lalias;
} og_graph;

enum { OG_NODE2VEC = 1, OG_METAPATH = 2, OG_SECOND_PR = 3 };
typedef struct {
    int32_t kind;
    int32_t weighted;
    float p, q;          /* Node2Vec a, b */
    float gamma;         /* second-order PageRank */
    int32_t schema_len;  /* MetaPath */
    uint8_t schema[64];
} og_logic;

typedef struct {
    float rho;           /* EdgeCost_RJS / EdgeCost_RVS */
    int32_t d_lo;        /* degree below which eRVS is always used */
    int32_t rjs_cap;     /* eRJS trials before falling back to eRVS */
    int32_t lanes;       /* eRVS lanes P */
    int32_t jump;        /* 1: Eq. (jump); 0: a key for every item */
    float bound_scale;   /* multiplies the eRJS bound (>= 1 keeps it a bound) */
    int32_t bound;       /* 0: max(w) * h_MAX (Section 3.3); 1: Node2Vec split bound; 2: split and
                            member board, the smaller per step */
    int32_t proposal;    /* 0: uniform eRJS proposals (Section 3.3); 1: proportional to h; 2: as 1,
                            and MetaPath proposes within the wanted label's group (og_build_label_alias) */
    int32_t hub_deg;     /* rows of at least this degree run eRVS with hub_lanes lanes (0: never) */
    int32_t hub_lanes;   /* P for those rows */
    int32_t rvs_share;   /* 1: after each eRVS round with a jump event the lanes take the largest
                            threshold among them, their skips rescaled (rvs_sample) */
} og_plan;

/* OG_RANDOM_SELECT and OG_DEGREE_SELECT are the two selection policies the paper compares
 * its cost model against (Section 6, sensitivity on selection strategy): a fair coin per
 * step (draw tag 4), and eRVS below a degree threshold (plan.d_lo, 1K in the paper) with
 * eRJS above it. */
enum { OG_AUTO = 0, OG_RVS_ONLY = 1, OG_RJS_ONLY = 2, OG_ITS = 3, OG_RANDOM_SELECT = 4, OG_DEGREE_SELECT = 5 };

/* Per-node preprocessing: h_MAX is the row maximum of h; h_SUM is the row sum of h,
 * accumulated in double and rounded once to float32 (Section 4.2, preprocess()). */
void og_preprocess(const og_graph *g, float *hmax, float *hsum)
{
    #pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t v = 0; v < g->nv; ++v) {
        float mx = 0.0f;
        double sm = 0.0;
        for (int64_t k = g->row_ptr[v]; k < g->row_ptr[v + 1]; ++k) {
            float hv = g->h ? g->h[k] : 1.0f;
            if (hv > mx) mx = hv;
            sm += (double)hv;
        }
        hmax[v] = mx;
        hsum[v] = (float)sm;
    }
}

/* Alias tables of the static weights h (Walker, "An efficient method for generating
 * discrete random variables with general distributions", ACM TOMS 1977), built with the
 * sweeping construction of Huebschle-Schneider and Sanders ("Parallel Weighted Random
 * Sampling", ESA 2019) in exact integer arithmetic, so that any correct execution of it,
 * sequential or parallel, yields the same table.
 *
 * Row v with n entries and row maximum h_MAX:
 *   q_k = floor(h_k / h_MAX * 2^32)   (the quotient in double, one rounding; 2^32 for
 *                                      every entry of an unweighted or all-zero row)
 *   Q   = sum q_k;  a bucket holds Q units, entry k brings a_k = q_k * n units;
 *   light entries have a_k < Q, heavy ones a_k >= Q.
 * The sweep walks the light entries in index order with a current heavy entry j (the
 * heavy entries in index order) holding a residual r, starting at r = a_j:
 *   - while r < Q, heavy j is spent: its bucket keeps r, its alias is the next heavy
 *     entry j', which first tops that bucket up: r = a_j' - (Q - r);
 *   - the light entry i keeps a_i with alias j, and r -= Q - a_i.
 * After the last light entry the remaining heavy entries are closed the same way (a
 * bucket that keeps a full Q is its own alias).  Every value stays below 2^63.
 * A bucket that keeps K units stores the threshold min(floor(K * 2^32 / Q), 2^32 - 1): a
 * proposal draws a 64-bit R, takes slot floor(R * n / 2^64) and keeps it when the high
 * 32 bits of the fraction (R * n mod 2^64) lie below the threshold, else takes its alias;
 * entry k then has probability q_k / Q, which is h_k / sum h up to the 2^-32 rounding of
 * q_k and of the thresholds. */
static uint32_t alias_threshold(uint64_t keep, uint64_t Q)
{
    const unsigned __int128 t = ((unsigned __int128)keep << 32) / Q;
    return t >= 0xFFFFFFFFu ? 0xFFFFFFFFu : (uint32_t)t;
}

/* The sweep over one sequence of n >= 1 values h[0..n) (NULL: all 1) with maximum hmax:
 * thr[k] and alias[k] (an index into the sequence) for each k. */
static void alias_sweep(const float *h, int64_t n, float hmax, uint32_t *thr, int32_t *alias)
{
    uint64_t *a = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    uint64_t Q = 0;
    for (int64_t k = 0; k < n; ++k) {
        const uint64_t q = (h && hmax > 0.0f) ? (uint64_t)floor(((double)h[k] / (double)hmax) * 4294967296.0)
                                              : (uint64_t)1 << 32;
        a[k] = q;
        Q += q;
    }
    for (int64_t k = 0; k < n; ++k) a[k] *= (uint64_t)n;
    int64_t j = 0;
    while (a[j] < Q) ++j; /* the first heavy entry (one exists: the a_k sum to n * Q) */
    uint64_t r = a[j];
    for (int64_t i = 0; i < n; ++i) {
        if (a[i] >= Q) continue; /* light entries only */
        while (r < Q) { /* a later heavy entry exists: the residuals of the heavy
                           entries cover every light entry's deficit exactly */
            int64_t jn = j + 1;
            while (jn < n - 1 && a[jn] < Q) ++jn;
            thr[j] = alias_threshold(r, Q);
            alias[j] = (int32_t)jn;
            r = a[jn] - (Q - r);
            j = jn;
        }
        thr[i] = alias_threshold(a[i], Q);
        alias[i] = (int32_t)j;
        r -= Q - a[i];
    }
    for (;;) { /* close the remaining heavy entries */
        int64_t jn = j + 1;
        while (jn < n && a[jn] < Q) ++jn;
        thr[j] = alias_threshold(r, Q);
        alias[j] = (int32_t)((r < Q && jn < n) ? jn : j);
        if (jn >= n) break;
        r = a[jn] - (Q - r);
        j = jn;
    }
    if (OG_MUTANT == 8)
        for (int64_t k = 0; k < n; ++k) thr[k] = 0xFFFFFFFFu;
    free(a);
}

void og_build_alias(const og_graph *g, uint32_t *thr, int32_t *alias)
{
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t v = 0; v < g->nv; ++v) {
        const int64_t b = g->row_ptr[v], n = g->row_ptr[v + 1] - b;
        if (n == 0) continue;
        float hmax = 0.0f;
        for (int64_t k = 0; k < n; ++k)
            if (g->h && g->h[b + k] > hmax) hmax = g->h[b + k];
        alias_sweep(g->h ? g->h + b : NULL, n, hmax, thr + b, alias + b);
    }
}

/* Label groups for label-conditioned proposals (plan.proposal = 2, MetaPath; an extension,
 * not in the paper).  Row v's entries are taken in (label, row position) order; the entries
 * of label l form group (v, l), whose first grouped position is lrow[v * nlab + l] (so that
 * lrow[v * nlab] = row_ptr[v] and lrow[nv * nlab] = ne).  lperm gives each grouped
 * position's row offset, and each group gets the alias table of its own h values by the
 * sweep above (its maximum as h_MAX; lalias indexes the group).  A MetaPath step that
 * wants label l then proposes from group (v, l) alone: every proposal has the wanted label
 * and probability h / (sum of h over the group), so one trial samples the step.  Returns
 * -1 if a label is >= nlab. */
int og_build_label_alias(const og_graph *g, int32_t nlab, int64_t *lrow, int32_t *lperm, uint32_t *lthr,
                         int32_t *lalias)
{
    for (int64_t k = 0; k < g->ne; ++k)
        if (g->label[k] >= nlab) return -1;
    int bad = 0;
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t v = 0; v < g->nv; ++v) {
        const int64_t b = g->row_ptr[v], n = g->row_ptr[v + 1] - b;
        int64_t pos = b;
        float *hg = (float *)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
        for (int32_t l = 0; l < nlab; ++l) {
            lrow[v * nlab + l] = pos;
            const int64_t g0 = pos;
            float hmax = 0.0f;
            for (int64_t k = 0; k < n; ++k) {
                if (g->label[b + k] != l) continue;
                lperm[pos] = (int32_t)k;
                hg[pos - g0] = g->h ? g->h[b + k] : 1.0f;
                if (hg[pos - g0] > hmax) hmax = hg[pos - g0];
                ++pos;
            }
            if (pos > g0) alias_sweep((g->h && OG_MUTANT != 13) ? hg : NULL, pos - g0, hmax, lthr + g0, lalias + g0);
        }
        if (pos != b + n) bad = 1;
        free(hg);
    }
    lrow[g->nv * nlab] = g->ne;
    return bad ? -1 : 0;
}
/* ------------------------------------------------------------------ one step */
typedef struct {
    const og_graph *g;
    const float *hmax, *hsum;
    const og_logic *lg;
    const og_plan *pl;
    int strategy;
    uint64_t seed;
} og_ctx;

typedef struct {
    float margin;   /* smallest relative gap of a float comparison in this step */
    int kind;       /* 0 eRVS, 1 eRJS accepted, 2 eRJS capped then eRVS, 3 ITS, -1 terminated */
    int trials;
    int triggers;
    double bytes;   /* algorithmic bytes of this step */
} og_info;

static void note_margin(og_info *info, float a, float b)
{
    float d = fabsf(a - b), m = fmaxf(fabsf(a), fabsf(b));
    float r = m > 0.0f ? d / m : 0.0f;
    if (r < info->margin) info->margin = r;
}

static int cmp_i32(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

static int is_neighbour(const og_graph *g, int32_t prev, int32_t u)
{
    int64_t b = g->row_ptr[prev], n = g->row_ptr[prev + 1] - b;
    return n > 0 && bsearch(&u, g->col + b, (size_t)n, sizeof(int32_t), cmp_i32) != NULL;
}

static int ceil_log2_plus1(int64_t m) /* ceil(log2(m + 1)): probes of a binary search */
{
    int c = 0;
    while (((int64_t)1 << c) < m + 1) ++c;
    return c;
}

/* The two values of the second-order PageRank weight at a step with d(v) = dv and
 * d(v') = dvp, in float32 in the order Eq. (2ndpr) writes them: in = for u in N(v'),
 * out = otherwise. */
static void second_pr_weights(const og_logic *lg, int64_t dv, int64_t dvp, float *in, float *out)
{
    const float a = 1.0f - lg->gamma;
    const float t1 = a / (float)dv;
    const float t2 = lg->gamma / (float)(OG_MUTANT == 7 ? dv : dvp);
    const float md = (float)(dv > dvp ? dv : dvp);
    *in = (t1 + t2) * md;
    *out = t1 * md;
}

/* Workload weight w(v, u) for the edge at CSR position k (u = col[k]) at step j, where
 * v has degree dv and the previous vertex prev has degree dvp. */
static float workload_weight(const og_ctx *cx, int64_t k, int j, int32_t prev, int64_t dv, int64_t dvp)
{
    const og_logic *lg = cx->lg;
    if (lg->kind == OG_SECOND_PR) {
        if (j == 0) return 1.0f;                     /* no previous vertex yet */
        float in, out;
        second_pr_weights(lg, dv, dvp, &in, &out);
        int32_t u = cx->g->col[k];
        return (u != prev && is_neighbour(cx->g, prev, u)) ? in : out; /* dist(v', u) = 1 or not */
    }
    if (lg->kind == OG_NODE2VEC) {
        if (j == 0) return 1.0f;                     /* no previous vertex yet */
        int32_t u = cx->g->col[k];
        if (u == prev) return 1.0f / (OG_MUTANT == 1 ? lg->q : lg->p); /* dist(v', u) = 0 */
        if (is_neighbour(cx->g, prev, u)) return 1.0f; /* dist(v', u) = 1 */
        return 1.0f / lg->q;                         /* dist(v', u) = 2 */
    }
    /* MetaPath: schema repeated along the walk */
    return cx->g->label[k] == lg->schema[j % lg->schema_len] ? 1.0f : 0.0f;
}

static float transition_weight(const og_ctx *cx, int64_t k, int j, int32_t prev, int64_t dv, int64_t dvp)
{
    float w = workload_weight(cx, k, j, prev, dv, dvp);
    if (cx->lg->weighted && cx->g->h) return w * cx->g->h[k];
    return w;
}

/* max over the workload's return values, and their mean (Section 4.2 helpers) */
static float w_max(const og_logic *lg, int j, int64_t dv, int64_t dvp)
{
    if (lg->kind == OG_NODE2VEC && j > 0) return fmaxf(fmaxf(1.0f / lg->p, 1.0f), 1.0f / lg->q);
    if (lg->kind == OG_SECOND_PR && j > 0) {
        float in, out;
        second_pr_weights(lg, dv, dvp, &in, &out);
        return fmaxf(in, out);
    }
    return 1.0f;
}

static float w_avg(const og_logic *lg, int j, int64_t dv, int64_t dvp)
{
    if (lg->kind == OG_SECOND_PR) {
        if (j == 0) return 1.0f;
        float in, out;
        second_pr_weights(lg, dv, dvp, &in, &out);
        return (in + out) / 2.0f;
    }
    if (lg->kind == OG_NODE2VEC) {
        if (j == 0) return 1.0f;
        return ((1.0f / lg->p + 1.0f) + 1.0f / lg->q) / (OG_MUTANT == 10 ? 2.0f : 3.0f);
    }
    return (1.0f + 0.0f) / 2.0f;
}

static double bytes_per_item(const og_ctx *cx)
{
    double b = 4.0;                                   /* col */
    if (cx->lg->weighted && cx->g->h) b += cx->g->h8 ? 1.0 : 4.0; /* h: float or 8-bit code */
    if (cx->lg->kind == OG_METAPATH) b += 1.0;        /* label */
    return b;
}

/* One eRVS lane: its best key lk (a logarithm) at item li, its threshold thr (the key
 * to beat), and the skip of Eq. (jump): the item whose running weight S passes T draws. */
typedef struct {
    float lk, thr, T, S;
    int64_t li;
} og_lane;

/* Item i of a lane's scan (Section 3.2, Eq. (jump)): add its weight to S; where S passes
 * T the item gets a key conditioned to beat thr, u' ~ U(exp(thr)^w~, 1), i.e.
 * ln u' = log1p(expm1(w~ * thr) * V), which becomes the lane's key and threshold, and a
 * new skip T = ln(r) / thr starts.  Returns 1 when a key was drawn. */
static int rvs_item(const og_ctx *cx, uint32_t w, int j, int32_t prev, int64_t base, int64_t deg, int64_t dvp,
                    int64_t i, og_lane *ln, og_info *info)
{
    uint32_t x[4];
    float wt = transition_weight(cx, base + i, j, prev, deg, dvp);
    ln->S = ln->S + wt;
    if (ln->T > 0.0f && ln->T < INFINITY) note_margin(info, ln->S, ln->T);
    if (!(ln->S > ln->T)) return 0;
    draw(cx->seed, w, (uint32_t)j, (uint32_t)i, 1, x);
    float a = wt * ln->thr;
    float m1 = expm1_f(a);
    float z = m1 * og_uniform(x[0]);
    float L = log1p_f(z);
    if (OG_MUTANT == 2) L = ln_f(og_uniform(x[0]));
    ln->lk = L / wt;
    ln->li = i;
    ln->thr = ln->lk;
    if (OG_MUTANT != 3) ln->S = 0.0f;
    ln->T = ln->thr >= 0.0f ? INFINITY : ln_f(og_uniform(x[1])) / ln->thr;
    info->triggers++;
    return 1;
}

/* eRVS over the row of `cur`, Section 3.2.  Returns the CSR offset within the row or -1. */
static int64_t rvs_sample(const og_ctx *cx, uint32_t w, int j, int32_t prev, int64_t base, int64_t deg,
                          int64_t dvp, og_info *info)
{
    /* P: the plan's lanes, or hub_lanes on a row of degree >= hub_deg */
    const int64_t P = (cx->pl->hub_deg > 0 && deg >= cx->pl->hub_deg) ? cx->pl->hub_lanes : cx->pl->lanes;
    uint32_t x[4];

    if (!cx->pl->jump) {
        /* Exponential keys without jumps (Section 3.2): every item of positive weight gets
           the key u_i^(1/w~_i), here its logarithm ln(u_i) / w~_i (the logarithm is
           increasing, so the largest key is the same item); the sample is the item of the
           largest key, the larger index among equal keys.  Items of weight 0 are not
           eligible; with none eligible the walk ends. */
        float best = -INFINITY;
        int64_t best_i = -1;
        for (int64_t i = 0; i < deg; ++i) {
            float wt = transition_weight(cx, base + i, j, prev, deg, dvp);
            if (!(wt > 0.0f)) continue;
            draw(cx->seed, w, (uint32_t)j, (uint32_t)i, 1, x);
            float key = ln_f(og_uniform(x[0])) / wt;
            if (best_i >= 0) note_margin(info, key, best);
            int wins = best_i < 0 || key > best || (key == best && i > best_i);
            if (wins) { best = key; best_i = i; }
        }
        return best_i;
    }

    /* Round 0: lane l keys its first item l; the maximum is shared by all lanes. */
    const int64_t n0 = deg < P ? deg : P;
    og_lane *ln = (og_lane *)malloc(sizeof(og_lane) * (size_t)n0);
    float lkg = -INFINITY;
    for (int64_t l = 0; l < n0; ++l) {
        float wt = transition_weight(cx, base + l, j, prev, deg, dvp);
        draw(cx->seed, w, (uint32_t)j, (uint32_t)l, 1, x);
        ln[l].lk = wt > 0.0f ? ln_f(og_uniform(x[0])) / wt : -INFINITY;
        ln[l].li = l;
        ln[l].T = og_uniform(x[1]); /* the threshold draw, until lkg is known */
        if (ln[l].lk > lkg) lkg = ln[l].lk;
    }
    for (int64_t l = 0; l < n0; ++l) {
        ln[l].thr = lkg;
        ln[l].T = lkg == -INFINITY ? 0.0f : (lkg >= 0.0f ? INFINITY : ln_f(ln[l].T) / lkg);
        ln[l].S = 0.0f;
    }

    if (!cx->pl->rvs_share) {
        /* Each lane scans items l+P, l+2P, ... on its own thresholds (Eq. (jump)). */
        for (int64_t l = 0; l < n0; ++l)
            for (int64_t i = l + P; i < deg; i += P)
                rvs_item(cx, w, j, prev, base, deg, dvp, i, &ln[l], info);
    } else {
        /* Round r holds items rP .. rP+P-1, lane l item rP+l.  After a round in which some
           lane drew a key, every lane whose threshold lies below the largest one, thr_g,
           takes thr_g: its remaining skip T - S is exponential with rate -thr (memoryless:
           no item since its last draw has passed it), and scaled by thr / thr_g it is
           exponential with rate -thr_g, the skip towards the first item whose key beats
           thr_g.  Keys below thr_g cannot win the final argmax, so no item loses its
           chance; only fewer keys are drawn.  A lane without a threshold (thr = -inf,
           every item so far of weight 0) keeps T = 0. */
        for (int64_t r0 = P; r0 < deg; r0 += P) {
            int drew = 0;
            for (int64_t l = 0; l < n0 && r0 + l < deg; ++l)
                drew |= rvs_item(cx, w, j, prev, base, deg, dvp, r0 + l, &ln[l], info);
            if (!drew) continue;
            float g = -INFINITY;
            for (int64_t l = 0; l < n0; ++l)
                if (ln[l].thr > g) g = ln[l].thr;
            for (int64_t l = 0; l < n0; ++l) {
                if (!(ln[l].thr > -INFINITY) || !(ln[l].thr < g)) continue;
                if (OG_MUTANT != 15) {
                    ln[l].T = g >= 0.0f ? INFINITY
                                        : (OG_MUTANT == 14 ? ((ln[l].T - ln[l].S) * g) / ln[l].thr
                                                           : ((ln[l].T - ln[l].S) * ln[l].thr) / g);
                    ln[l].S = 0.0f;
                }
                ln[l].thr = g;
            }
        }
    }

    /* lexicographic maximum over (key, index): larger index wins ties */
    float best = -INFINITY, second = -INFINITY;
    int64_t best_i = -1;
    for (int64_t l = 0; l < n0; ++l) {
        const float lk = ln[l].lk;
        const int64_t li = ln[l].li;
        if (lk > best || (lk == best && li > best_i)) {
            second = best;
            best = lk;
            best_i = li;
        } else if (lk > second) {
            second = lk;
        }
    }
    if (best > -INFINITY && second > -INFINITY) note_margin(info, best, second);
    free(ln);
    return best > -INFINITY ? best_i : -1;
}

/* eRJS, Section 3.3.  Returns the row offset, or -2 when the cap is reached.  With
 * E > 0 (split bound) a trial first decides between the extra column of height E,
 * owned by the return edge at row offset ret, and the deg regular columns of height B. */
static int64_t rjs_sample(const og_ctx *cx, uint32_t w, int j, int32_t prev, int64_t base, int64_t deg,
                          int64_t dvp, float B, float E, int64_t ret, float area, int hprop, og_info *info)
{
    uint32_t x[4];
    const og_logic *lg = cx->lg;
    for (int t = 0; t < cx->pl->rjs_cap; ++t) {
        draw(cx->seed, w, (uint32_t)j, (uint32_t)t, 0, x);
        info->trials++;
        if (E > 0.0f) {
            float z = og_uniform(x[3]) * area;
            note_margin(info, z, E);
            if (z < E) return ret;
        }
        uint64_t R = ((uint64_t)x[1] << 32) | x[0];
        const unsigned __int128 P = (unsigned __int128)R * (unsigned __int128)(uint64_t)deg;
        int64_t idx = (int64_t)(P >> 64);
        if (OG_MUTANT == 4 && deg > 1) idx = (int64_t)(((unsigned __int128)R * (unsigned __int128)(uint64_t)(deg - 1)) >> 64);
        if (hprop) {
            /* alias coin: the high 32 bits of the fraction against the slot's threshold */
            const uint32_t f = (uint32_t)((uint64_t)P >> 32);
            if (!(f < cx->g->alias_thr[base + idx])) idx = cx->g->alias_idx[base + idx];
        }
        /* uniform proposals test U * B against w~; h-proportional ones U * B against w */
        float wt = hprop ? workload_weight(cx, base + idx, j, prev, deg, dvp)
                         : transition_weight(cx, base + idx, j, prev, deg, dvp);
        float y = og_uniform(x[2]) * B;
        /* bytes: the proposed edge, the alias slot's threshold and second candidate
           (h-proportional), and the binary search of N(v') that decides u in N(v')
           (Node2Vec, second-order PageRank after the first step), charged on every trial */
        info->bytes += bytes_per_item(cx) + (hprop ? 12.0 : 0.0);
        if ((lg->kind == OG_NODE2VEC || lg->kind == OG_SECOND_PR) && j > 0)
            info->bytes += 4.0 * ceil_log2_plus1(dvp);
        if (y < wt) return idx;
    }
    return -2;
}

/* Offset of u in the sorted row of v, or -1. */
static int64_t row_find(const og_graph *g, int32_t v, int32_t u)
{
    int64_t b = g->row_ptr[v], n = g->row_ptr[v + 1] - b;
    const int32_t *p = n > 0 ? (const int32_t *)bsearch(&u, g->col + b, (size_t)n, sizeof(int32_t), cmp_i32) : NULL;
    return p ? (int64_t)(p - (g->col + b)) : -1;
}

/* eRJS on the member board (plan.bound = 2).  z = U(x3) * A picks the return column
 * [0, E), the member region [E, E + R) or the regular columns; a member-region trial takes
 * x = N(v')[floor(R64 * d(v') / 2^64)] and keeps it iff x != v', x in N(v) and
 * U(x2) * h_MAX < h(v, x); a regular trial proposes as usual (uniform or h-proportional)
 * and keeps u with min(w_u, w_oth) / w_oth of the usual test, members counted at w_oth. */
static int64_t rjs_sample_member(const og_ctx *cx, uint32_t w, int j, int32_t prev, int32_t cur, int64_t base,
                                 int64_t deg, int64_t dvp, float woth, float wret, float hm, float E, float R,
                                 float area, int64_t ret, int hprop, og_info *info)
{
    const og_graph *g = cx->g;
    const int64_t pbase = g->row_ptr[prev];
    uint32_t x[4];
    const float zm = E + R;
    for (int t = 0; t < cx->pl->rjs_cap; ++t) {
        draw(cx->seed, w, (uint32_t)j, (uint32_t)t, 0, x);
        info->trials++;
        const float z = og_uniform(x[3]) * area;
        if (E > 0.0f) {
            note_margin(info, z, E);
            if (z < E) return ret;
        }
        const uint64_t R64 = ((uint64_t)x[1] << 32) | x[0];
        note_margin(info, z, zm);
        if (z < zm) {
            const int32_t xv = g->col[pbase + (int64_t)(((unsigned __int128)R64 * (unsigned __int128)(uint64_t)dvp) >> 64)];
            /* bytes: x, a binary search of N(v) for it, and h(v, x) */
            info->bytes += 4.0 + 4.0 * ceil_log2_plus1(deg) + (cx->lg->weighted && g->h ? 4.0 : 0.0);
            if (xv == prev) continue;
            const int64_t pos = row_find(g, cur, xv);
            if (pos < 0) continue;
            const float hx = (cx->lg->weighted && g->h) ? g->h[base + pos] : 1.0f;
            const float y = og_uniform(x[2]) * hm;
            if (y < hx || OG_MUTANT == 9) return pos;
            continue;
        }
        const unsigned __int128 P = (unsigned __int128)R64 * (unsigned __int128)(uint64_t)deg;
        int64_t idx = (int64_t)(P >> 64);
        if (hprop) {
            const uint32_t f = (uint32_t)((uint64_t)P >> 32);
            if (!(f < g->alias_thr[base + idx])) idx = g->alias_idx[base + idx];
        }
        info->bytes += bytes_per_item(cx) + (hprop ? 12.0 : 0.0);
        const float wu = g->col[base + idx] == prev ? fminf(wret, woth) : woth;
        const float hu = (!hprop && cx->lg->weighted && g->h) ? g->h[base + idx] : 1.0f;
        const float y = og_uniform(x[2]) * (hprop ? woth : woth * hm);
        if (y < wu * hu) return idx;
    }
    return -2;
}

/* Inverse transform sampling over the exact weights (plain CPU sampler). */
static int64_t its_sample(const og_ctx *cx, uint32_t w, int j, int32_t prev, int64_t base, int64_t deg,
                          int64_t dvp, og_info *info)
{
    double *cum = (double *)malloc(sizeof(double) * (size_t)deg);
    double run = 0.0;
    for (int64_t i = 0; i < deg; ++i) {
        run += (double)transition_weight(cx, base + i, j, prev, deg, dvp);
        cum[i] = run;
    }
    int64_t res = -1;
    if (run > 0.0) {
        uint32_t x[4];
        draw(cx->seed, w, (uint32_t)j, 0, 3, x);
        double u = ((double)(x[0] >> 5) * 67108864.0 + (double)(x[1] >> 6)) * 0x1p-53;
        double target = u * run;
        /* first item whose cumulative weight exceeds the target; it always has
           a positive weight because the cumulative sum is flat over zero weights */
        int64_t lo = 0, hi = deg - 1;
        while (lo < hi) {
            int64_t mid = (lo + hi) / 2;
            if (cum[mid] > target) hi = mid; else lo = mid + 1;
        }
        res = lo;
    }
    info->bytes += (double)deg * bytes_per_item(cx);
    free(cum);
    return res;
}

/* One transition from state (prev, cur, j) of walker w.  Returns the next vertex or -1. */
int32_t og_step(const og_ctx *cx, uint32_t w, int j, int32_t prev, int32_t cur, og_info *info)
{
    const og_graph *g = cx->g;
    const og_logic *lg = cx->lg;
    info->margin = FLT_MAX;
    info->kind = -1;
    info->trials = 0;
    info->triggers = 0;
    info->bytes = OG_MUTANT == 12 ? 8.0 : 16.0; /* row_ptr[cur], row_ptr[cur + 1]: two 8-byte offsets */
    const int64_t base = g->row_ptr[cur], deg = g->row_ptr[cur + 1] - base;
    if (deg == 0) return -1;

    const int64_t dvp = j > 0 ? g->row_ptr[prev + 1] - g->row_ptr[prev] : 0; /* d(v') */
    const int weighted = lg->weighted && g->h;

    /* label-conditioned proposals (plan.proposal = 2, MetaPath): the step's eRJS draws one
       proposal from the group of the wanted label, which it always keeps; its eRJS cost is
       one trial against deg for eRVS in Eq. (runtime).  A step whose group is empty, or
       whose group has only zero weights, ends the walk (no neighbour has positive weight). */
    if (lg->kind == OG_METAPATH && cx->pl->proposal == 2 && cx->strategy != OG_ITS) {
        const int want = lg->schema[j % lg->schema_len];
        info->bytes += 8.0; /* the group's first and last position */
        const int64_t g0 = want < g->nlab ? g->lrow[cur * g->nlab + want] : 0;
        const int64_t n = want < g->nlab ? g->lrow[cur * g->nlab + want + 1] - g0 : 0;
        if (n == 0) return -1;
        int use_rjs = 0;
        if (cx->strategy == OG_RJS_ONLY) {
            use_rjs = 1;
        } else if (cx->strategy == OG_AUTO) {
            if (deg >= cx->pl->d_lo) {
                note_margin(info, cx->pl->rho, (float)deg);
                use_rjs = cx->pl->rho < (float)deg; /* a tie goes to eRVS */
            }
        } else if (cx->strategy == OG_RANDOM_SELECT) {
            uint32_t x[4];
            draw(cx->seed, w, (uint32_t)j, 0, 4, x);
            use_rjs = og_uniform(x[0]) < 0.5f;
        } else if (cx->strategy == OG_DEGREE_SELECT) {
            use_rjs = deg >= cx->pl->d_lo;
        }
        int64_t off;
        if (use_rjs) {
            uint32_t x[4];
            draw(cx->seed, w, (uint32_t)j, 0, 0, x);
            info->trials = 1;
            const uint64_t R = ((uint64_t)x[1] << 32) | x[0];
            const unsigned __int128 P = (unsigned __int128)R * (unsigned __int128)(uint64_t)n;
            int64_t t = (int64_t)(P >> 64);
            const uint32_t f = (uint32_t)((uint64_t)P >> 32);
            if (!(f < g->lthr[g0 + t])) t = g->lalias[g0 + t];
            off = g->lperm[g0 + t];
            info->bytes += bytes_per_item(cx) + 12.0;
            if (weighted && !(g->h[base + off] > 0.0f)) return -1; /* the group's weights are all 0 */
            info->kind = 1;
        } else {
            info->kind = 0;
            info->bytes += (double)deg * bytes_per_item(cx);
            off = rvs_sample(cx, w, j, prev, base, deg, dvp, info);
            if (off < 0) {
                info->kind = -1;
                return -1;
            }
        }
        return g->col[base + off];
    }
    const float hm = (weighted && OG_MUTANT != 5) ? cx->hmax[cur] : 1.0f;
    const float hs = weighted ? cx->hsum[cur] : (float)deg;
    /* h-proportional proposals: the eRJS test compares U * B with w (not w~), so B bounds
       the workload weights alone */
    const int hprop = cx->pl->proposal >= 1 && weighted;
    const float hB = hprop ? 1.0f : hm;
    float B = (w_max(lg, j, deg, dvp) * hB) * cx->pl->bound_scale; /* upper bound of max w~ (or w) */
    const float Shat = w_avg(lg, j, deg, dvp) * hs;                /* estimate of sum w~ */

    /* split bound: regular height over the non-return weights, extra column for the
       return edge's excess (w~ret of the edge cur -> prev, 0 if there is none) */
    const int split = (cx->pl->bound == 1 || cx->pl->bound == 2) && lg->kind == OG_NODE2VEC && j > 0;
    float E = 0.0f;
    int64_t ret = -1;
    if (split) {
        B = (fmaxf(1.0f, 1.0f / lg->q) * hB) * cx->pl->bound_scale;
        for (int64_t i = 0; i < deg; ++i)
            if (g->col[base + i] == prev) ret = i;
        if (ret >= 0) {
            float wret = transition_weight(cx, base + ret, j, prev, deg, dvp);
            /* the return edge's column has width 1 (uniform) or h(v, prev) (h-proportional) */
            float cell = hprop ? B * g->h[base + ret] : B;
            E = OG_MUTANT == 6 ? wret : fmaxf(0.0f, wret - cell);
        }
    }
    /* area of the proposal board: deg columns of height B (uniform) or total width
       sum h = h_SUM at height B (h-proportional), plus the return edge's extra column */
    float area = hprop ? B * hs + E : (float)deg * B + E;

    /* member board: w_mem on N(v') above w_oth elsewhere; used when its area is smaller */
    int member = 0;
    float woth = 0.0f, wmem = 0.0f, wret = 0.0f, Em = 0.0f, Rm = 0.0f;
    if (cx->pl->bound == 2 && j > 0 && dvp > 0 && (lg->kind == OG_NODE2VEC || lg->kind == OG_SECOND_PR)) {
        if (lg->kind == OG_NODE2VEC) {
            woth = 1.0f / lg->q;
            wmem = 1.0f;
            wret = 1.0f / lg->p;
        } else {
            second_pr_weights(lg, deg, dvp, &wmem, &woth);
            wret = woth;
        }
        if (wmem > woth) {
            const float hmx = weighted ? cx->hmax[cur] : 1.0f;
            const float areg = hprop ? woth * hs : ((float)deg * woth) * hmx;
            Rm = ((wmem - woth) * hmx) * (float)dvp;
            if (lg->kind == OG_NODE2VEC && ret < 0)
                for (int64_t i = 0; i < deg; ++i)
                    if (g->col[base + i] == prev) ret = i;
            if (lg->kind == OG_NODE2VEC && ret >= 0) {
                const float hr = weighted ? g->h[base + ret] : 1.0f;
                Em = fmaxf(0.0f, transition_weight(cx, base + ret, j, prev, deg, dvp) - woth * hr);
            }
            const float am = (areg + Rm) + Em;
            if (am < area) {
                member = 1;
                area = am;
            }
        }
    }

    int use_rjs = 0;
    if (cx->strategy == OG_RJS_ONLY) {
        use_rjs = 1;
        if (weighted) info->bytes += 4.0;
    } else if (cx->strategy == OG_AUTO) {
        if (weighted) info->bytes += 8.0;
        if (deg >= cx->pl->d_lo) {
            /* Eq. (runtime) per edge; with the split or h-proportional proposals the
               expected-trial cost is area / S, compared against the eRVS cost deg */
            const int board = split || hprop || member;
            float lhs = board ? cx->pl->rho * area : cx->pl->rho * B;
            float rhs = board ? (float)deg * Shat : Shat;
            note_margin(info, lhs, rhs);
            use_rjs = OG_MUTANT == 11 ? !(lhs < rhs) : lhs < rhs; /* a tie goes to eRVS */
        }
    } else if (cx->strategy == OG_RANDOM_SELECT) {
        if (weighted) info->bytes += 4.0;
        uint32_t x[4];
        draw(cx->seed, w, (uint32_t)j, 0, 4, x);
        use_rjs = og_uniform(x[0]) < 0.5f;
    } else if (cx->strategy == OG_DEGREE_SELECT) {
        if (weighted) info->bytes += 4.0;
        use_rjs = deg >= cx->pl->d_lo;
    }

    int64_t off;
    if (cx->strategy == OG_ITS) {
        info->kind = 3;
        off = its_sample(cx, w, j, prev, base, deg, dvp, info);
    } else {
        off = -2;
        /* h-proportional proposals need some positive h; a row without goes to eRVS */
        if (use_rjs && !(hprop && !(hs > 0.0f))) {
            off = member ? rjs_sample_member(cx, w, j, prev, cur, base, deg, dvp, woth, wret,
                                             weighted ? cx->hmax[cur] : 1.0f, Em, Rm, area, ret, hprop, info)
                         : rjs_sample(cx, w, j, prev, base, deg, dvp, B, E, ret, area, hprop, info);
            info->kind = 1;
        }
        if (off == -2) {
            info->kind = use_rjs ? 2 : 0;
            info->bytes += (double)deg * bytes_per_item(cx);
            if ((lg->kind == OG_NODE2VEC || lg->kind == OG_SECOND_PR) && j > 0) {
                int64_t pdeg = dvp;
                double stage = 4.0 * (double)pdeg;
                double search = 4.0 * (double)deg * ceil_log2_plus1(pdeg);
                info->bytes += stage < search ? stage : search;
            }
            off = rvs_sample(cx, w, j, prev, base, deg, dvp, info);
        }
    }
    if (off < 0) {
        info->kind = -1;
        return -1;
    }
    return g->col[base + off];
}

/* ------------------------------------------------------------------ walks */
/* counters: 0 steps, 1 eRJS accepted, 2 eRVS, 3 eRJS capped -> eRVS, 4 eRJS trials,
 *           5 eRVS jump triggers, 6 walks ended early, 7 algorithmic bytes,
 *           8 steps with margin < 1e-6 */
enum { OG_NCOUNTERS = 9 };

/*
 * Free-running walks.  Walker i starts at starts[i], uses RNG walker index
 * walker_ids[i] (or i) and writes paths[i*(L+1) .. i*(L+1)+L] (start, then the vertex
 * after each step, -1 after termination) and lengths[i] (steps taken).  margins and
 * kinds, when non-NULL, receive per-step diagnostics ([i*L + j]).  Returns 0, or -1
 * if a start vertex is out of range.
 */
int og_walk(const og_graph *g, const float *hmax, const float *hsum, const og_logic *lg, const og_plan *pl,
            int strategy, const int32_t *starts, const int64_t *walker_ids, int64_t n, int32_t L, uint64_t seed,
            int32_t *paths, int32_t *lengths, float *margins, int8_t *kinds, double *counters, int nthreads)
{
    for (int64_t i = 0; i < n; ++i)
        if (starts[i] < 0 || starts[i] >= g->nv) return -1;
    og_ctx cx = {g, hmax, hsum, lg, pl, strategy, seed};
    double c[OG_NCOUNTERS];
    memset(c, 0, sizeof(c));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    double c0 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0, c5 = 0, c6 = 0, c7 = 0, c8 = 0;
    #pragma omp parallel for schedule(dynamic, 16) reduction(+:c0,c1,c2,c3,c4,c5,c6,c7,c8)
    for (int64_t i = 0; i < n; ++i) {
        uint32_t w = (uint32_t)(walker_ids ? walker_ids[i] : i);
        int32_t *path = paths + i * (int64_t)(L + 1);
        int32_t cur = starts[i], prev = -1;
        int32_t len = 0;
        path[0] = cur;
        c7 += 4.0 + 4.0 * (L + 1) + 4.0; /* start read, path row, length */
        for (int j = 0; j < L; ++j) {
            og_info info;
            int32_t nxt = og_step(&cx, w, j, prev, cur, &info);
            if (margins) margins[i * (int64_t)L + j] = info.margin;
            if (kinds) kinds[i * (int64_t)L + j] = (int8_t)info.kind;
            c7 += info.bytes;
            c4 += info.trials;
            c5 += info.triggers;
            if (info.margin < 1e-6f) c8 += 1;
            if (nxt < 0) {
                c6 += 1;
                for (int r = j + 1; r < L; ++r) {
                    if (margins) margins[i * (int64_t)L + r] = FLT_MAX;
                    if (kinds) kinds[i * (int64_t)L + r] = -1;
                }
                break;
            }
            c0 += 1;
            if (info.kind == 1) c1 += 1;
            else if (info.kind == 0) c2 += 1;
            else if (info.kind == 2) c3 += 1;
            path[j + 1] = nxt;
            prev = cur;
            cur = nxt;
            len++;
        }
        for (int r = len + 1; r <= L; ++r) path[r] = -1;
        lengths[i] = len;
    }
    c[0] = c0; c[1] = c1; c[2] = c2; c[3] = c3; c[4] = c4; c[5] = c5; c[6] = c6; c[7] = c7; c[8] = c8;
    if (counters) memcpy(counters, c, sizeof(c));
    return 0;
}

/* Single transition for a given state (diagnostics and small tests); bytes receives the
 * step's algorithmic bytes (any output pointer may be NULL). */
int32_t og_step_once(const og_graph *g, const float *hmax, const float *hsum, const og_logic *lg,
                     const og_plan *pl, int strategy, uint64_t seed, uint32_t walker, int32_t j, int32_t prev,
                     int32_t cur, float *margin, int32_t *kind, int32_t *trials, double *bytes)
{
    og_ctx cx = {g, hmax, hsum, lg, pl, strategy, seed};
    og_info info;
    int32_t r = og_step(&cx, walker, j, prev, cur, &info);
    if (margin) *margin = info.margin;
    if (kind) *kind = info.kind;
    if (trials) *trials = info.trials;
    if (bytes) *bytes = info.bytes;
    return r;
}
