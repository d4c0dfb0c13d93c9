/*
 * Seeded synthetic graph inputs: R-MAT (Chakrabarti, Zhan, Faloutsos, "R-MAT: A
 * Recursive Model for Graph Mining", SDM 2004), symmetrised into a CSR with sorted,
 * de-duplicated rows, plus per-edge property weights and labels.
 *
 * This module produces inputs only.  It holds none of the random-walk arithmetic and
 * is shared by the CPU oracle and the GPU path purely as an input source.
 *
 * Determinism: every random quantity is a counter-based hash (SplitMix64 finaliser,
 * Steele, Lea, Flood, OOPSLA 2014) of (seed, index), so the output does not depend on
 * the thread count.  Weights and labels are hashed from the unordered vertex pair, so
 * both directions of an undirected edge carry the same values.
 *
 * Build: gcc -O3 -fopenmp -shared -fPIC rmat.c -o librmat.so
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static inline double u01(uint64_t x) { return (double)(x >> 11) * 0x1p-53; }

typedef struct {
    int64_t nv, ne;
    int64_t *row_ptr;
    int32_t *col;
    float *h;
    uint8_t *label;
} synth_csr;

/* One R-MAT draw: descend `scale` levels of the adjacency quadtree. */
static inline void rmat_edge(uint64_t seed, int64_t e, int scale, double a, double ab, double abc,
                             uint32_t *pu, uint32_t *pv)
{
    uint64_t s = mix64(seed ^ mix64((uint64_t)e));
    uint32_t u = 0, v = 0;
    for (int lvl = 0; lvl < scale; ++lvl) {
        double r = u01(mix64(s + (uint64_t)lvl * 0xD1B54A32D192ED03ull));
        uint32_t bu, bv;
        if (r < a)        { bu = 0; bv = 0; }
        else if (r < ab)  { bu = 0; bv = 1; }
        else if (r < abc) { bu = 1; bv = 0; }
        else              { bu = 1; bv = 1; }
        u = (u << 1) | bu;
        v = (v << 1) | bv;
    }
    *pu = u;
    *pv = v;
}

static int cmp_i32(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

void synth_free(synth_csr *g)
{
    if (!g) return;
    free(g->row_ptr); free(g->col); free(g->h); free(g->label);
    memset(g, 0, sizeof(*g));
}

/*
 * Fill per-edge property weights (uniform in [wlo, whi)) and labels (uniform in
 * 0..nlabels-1) for an existing CSR, hashed from the unordered pair.
 */
int synth_edge_props(int64_t nv, const int64_t *row_ptr, const int32_t *col, uint64_t seed,
                     float wlo, float whi, int nlabels, float *h, uint8_t *label)
{
    const uint64_t sw = mix64(seed ^ 0x5745494748545321ull);
    const uint64_t sl = mix64(seed ^ 0x4C4142454C532121ull);
    #pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t v = 0; v < nv; ++v) {
        for (int64_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) {
            uint64_t x = (uint64_t)v, y = (uint64_t)(uint32_t)col[k];
            uint64_t lo = x < y ? x : y, hi = x < y ? y : x;
            uint64_t pair = (hi << 32) | lo;
            if (h) {
                float w = (float)((double)wlo + ((double)whi - (double)wlo) * u01(mix64(sw ^ mix64(pair))));
                if (w >= whi) w = nextafterf(whi, wlo);
                if (w < wlo) w = wlo;
                h[k] = w;
            }
            if (label) label[k] = (uint8_t)(mix64(sl ^ mix64(pair)) % (uint64_t)(nlabels > 0 ? nlabels : 1));
        }
    }
    return 0;
}

/*
 * Generate an undirected R-MAT graph with 2^scale vertices from `ndraws` edge draws.
 * Self-loops are dropped, both directions are stored, duplicates are merged, vertex
 * ids are shuffled by a seeded permutation when `permute` is set, and each row is
 * sorted ascending.  Returns 0 on success, -1 on allocation failure.
 */
int synth_rmat(int scale, int64_t ndraws, double a, double b, double c, uint64_t seed, int permute,
               float wlo, float whi, int nlabels, int want_h, int want_label, synth_csr *out)
{
    memset(out, 0, sizeof(*out));
    const int64_t nv = (int64_t)1 << scale;
    const double ab = a + b, abc = a + b + c;

    uint32_t *perm = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)nv);
    int64_t *deg = (int64_t *)calloc((size_t)nv + 1, sizeof(int64_t));
    if (!perm || !deg) { free(perm); free(deg); return -1; }
    for (int64_t i = 0; i < nv; ++i) perm[i] = (uint32_t)i;
    if (permute) {
        /* Fisher-Yates with a counter-based stream */
        uint64_t sp = mix64(seed ^ 0x5045524D55544521ull);
        for (int64_t i = nv - 1; i > 0; --i) {
            uint64_t r = mix64(sp + (uint64_t)i);
            int64_t j = (int64_t)(((unsigned __int128)r * (unsigned __int128)(uint64_t)(i + 1)) >> 64);
            uint32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
        }
    }

    /* pass 1: degree count (both directions, self-loops dropped) */
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ndraws; ++e) {
        uint32_t u, v;
        rmat_edge(seed, e, scale, a, ab, abc, &u, &v);
        if (u == v) continue;
        uint32_t pu = perm[u], pv = perm[v];
        #pragma omp atomic
        deg[pu]++;
        #pragma omp atomic
        deg[pv]++;
    }
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nv + 1));
    if (!off) { free(perm); free(deg); return -1; }
    off[0] = 0;
    for (int64_t v = 0; v < nv; ++v) off[v + 1] = off[v] + deg[v];
    const int64_t raw = off[nv];
    int32_t *adj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(raw > 0 ? raw : 1));
    if (!adj) { free(perm); free(deg); free(off); return -1; }
    memcpy(deg, off, sizeof(int64_t) * (size_t)nv); /* reuse as fill cursor */

    /* pass 2: scatter */
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ndraws; ++e) {
        uint32_t u, v;
        rmat_edge(seed, e, scale, a, ab, abc, &u, &v);
        if (u == v) continue;
        uint32_t pu = perm[u], pv = perm[v];
        int64_t k1, k2;
        #pragma omp atomic capture
        k1 = deg[pu]++;
        #pragma omp atomic capture
        k2 = deg[pv]++;
        adj[k1] = (int32_t)pv;
        adj[k2] = (int32_t)pu;
    }
    free(perm);

    /* sort + dedup each row in place; deg[v] becomes the unique count */
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t v = 0; v < nv; ++v) {
        int32_t *r = adj + off[v];
        int64_t n = off[v + 1] - off[v];
        if (n > 1) qsort(r, (size_t)n, sizeof(int32_t), cmp_i32);
        int64_t m = 0;
        for (int64_t i = 0; i < n; ++i)
            if (m == 0 || r[m - 1] != r[i]) r[m++] = r[i];
        deg[v] = m;
    }

    int64_t *row_ptr = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nv + 1));
    if (!row_ptr) { free(deg); free(off); free(adj); return -1; }
    row_ptr[0] = 0;
    for (int64_t v = 0; v < nv; ++v) row_ptr[v + 1] = row_ptr[v] + deg[v];
    const int64_t ne = row_ptr[nv];
    int32_t *col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ne > 0 ? ne : 1));
    if (!col) { free(deg); free(off); free(adj); free(row_ptr); return -1; }
    #pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t v = 0; v < nv; ++v)
        memcpy(col + row_ptr[v], adj + off[v], sizeof(int32_t) * (size_t)deg[v]);
    free(adj); free(off); free(deg);

    float *h = NULL;
    uint8_t *label = NULL;
    if (want_h) h = (float *)malloc(sizeof(float) * (size_t)(ne > 0 ? ne : 1));
    if (want_label) label = (uint8_t *)malloc((size_t)(ne > 0 ? ne : 1));
    if ((want_h && !h) || (want_label && !label)) { free(h); free(label); free(col); free(row_ptr); return -1; }
    synth_edge_props(nv, row_ptr, col, seed, wlo, whi, nlabels, h, label);

    out->nv = nv; out->ne = ne; out->row_ptr = row_ptr; out->col = col; out->h = h; out->label = label;
    return 0;
}
