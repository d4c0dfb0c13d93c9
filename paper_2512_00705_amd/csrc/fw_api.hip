// C ABI of the sampler (include/flexiwalk.h): argument checks, device memory
// ownership, plan construction and kernel launches.  All sampling runs in
// fw_kernels.hip.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/flexiwalk.h"
#include "fw_device.h"
#include "fw_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok()
{
    g_err.clear();
    return FW_OK;
}

#define HIP_TRY(expr)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) return fail(FW_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

}  // namespace

struct fw_graph {
    int device = 0;
    int64_t nv = 0, ne = 0, max_deg = 0;
    int64_t *row_ptr = nullptr;
    int32_t *col = nullptr;
    float *h = nullptr;
    uint8_t *label = nullptr;
    uint2 *edges = nullptr;                 // {col, bits(h)} per entry
    uint4 *vrec = nullptr;                  // {start_lo, degree, bits(h_MAX), bits(h_SUM)} per vertex
    uint32_t *start_hi = nullptr;           // high row-start bits, only when ne >= 2^32
    unsigned long long *scratch = nullptr;  // [0] walker queue, [1] error flag (int)
    bool prepped = false;
};

static void graph_free(fw_graph *g)
{
    if (!g) return;
    (void)hipFree(g->row_ptr);
    (void)hipFree(g->col);
    (void)hipFree(g->h);
    (void)hipFree(g->label);
    (void)hipFree(g->edges);
    (void)hipFree(g->vrec);
    (void)hipFree(g->start_hi);
    (void)hipFree(g->scratch);
    delete g;
}

template <typename T>
static int dev_copy(T **dst, const T *src, int64_t count, int on_device)
{
    const size_t bytes = sizeof(T) * (size_t)(count > 0 ? count : 1);
    if (hipMalloc((void **)dst, bytes) != hipSuccess) {
        *dst = nullptr;
        return fail(FW_E_NOMEM, "hipMalloc of %zu bytes failed", bytes);
    }
    if (count > 0) HIP_TRY(hipMemcpy(*dst, src, sizeof(T) * (size_t)count,
                                     on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
    return FW_OK;
}

extern "C" {

const char *fw_last_error(void) { return g_err.c_str(); }

int fw_graph_create(const fw_csr *in, fw_graph **out)
{
    if (!in || !out) return fail(FW_E_INVALID, "fw_graph_create: null argument");
    if (in->nv < 0 || in->ne < 0) return fail(FW_E_INVALID, "fw_graph_create: negative size");
    if (in->nv >= ((int64_t)1 << 31)) return fail(FW_E_INVALID, "fw_graph_create: nv must be < 2^31");
    if (!in->row_ptr || (in->ne > 0 && !in->col))
        return fail(FW_E_INVALID, "fw_graph_create: row_ptr/col missing");

    fw_graph *g = new fw_graph();
    (void)hipGetDevice(&g->device);
    g->nv = in->nv;
    g->ne = in->ne;
    int rc;
    if ((rc = dev_copy(&g->row_ptr, in->row_ptr, in->nv + 1, in->on_device)) != FW_OK ||
        (rc = dev_copy(&g->col, in->col, in->ne, in->on_device)) != FW_OK ||
        (in->h && (rc = dev_copy(&g->h, in->h, in->ne, in->on_device)) != FW_OK) ||
        (in->label && (rc = dev_copy(&g->label, in->label, in->ne, in->on_device)) != FW_OK)) {
        graph_free(g);
        return rc;
    }
    const bool wide = g->ne >= ((int64_t)1 << 32);
    if (hipMalloc((void **)&g->edges, sizeof(uint2) * (size_t)(g->ne > 0 ? g->ne : 1)) != hipSuccess ||
        hipMalloc((void **)&g->vrec, sizeof(uint4) * (size_t)(g->nv > 0 ? g->nv : 1)) != hipSuccess ||
        (wide && hipMalloc((void **)&g->start_hi, sizeof(uint32_t) * (size_t)g->nv) != hipSuccess) ||
        hipMalloc((void **)&g->scratch, 4 * sizeof(unsigned long long)) != hipSuccess) {
        graph_free(g);
        return fail(FW_E_NOMEM, "fw_graph_create: hipMalloc failed");
    }

    // validate on the device: row pointers first (they bound every later access)
    unsigned long long *chk = g->scratch;  // [0] error bits, [1] max degree
    int host_err = 0;
    unsigned long long host_chk[2] = {0, 0};
    hipError_t e = hipMemset(chk, 0, 2 * sizeof(unsigned long long));
    if (e == hipSuccess) e = fw::launch_validate_rows(g->row_ptr, g->nv, g->ne, (int *)chk, nullptr);
    if (e == hipSuccess) e = hipMemcpy(host_chk, chk, sizeof(host_chk), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        graph_free(g);
        return fail(FW_E_DEVICE, "fw_graph_create: %s", hipGetErrorString(e));
    }
    host_err = (int)(host_chk[0] & 0xffffffffu);
    if (host_err != 0) {
        graph_free(g);
        return fail(FW_E_INVALID, "fw_graph_create: row_ptr must start at 0, end at ne and not decrease");
    }
    e = fw::launch_validate_edges(g->row_ptr, g->col, g->h, g->nv, (int *)chk, chk + 1, nullptr);
    if (e == hipSuccess) e = hipMemcpy(host_chk, chk, sizeof(host_chk), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        graph_free(g);
        return fail(FW_E_DEVICE, "fw_graph_create: %s", hipGetErrorString(e));
    }
    host_err = (int)(host_chk[0] & 0xffffffffu);
    if (host_err != 0) {
        graph_free(g);
        return fail(FW_E_INVALID,
                    "fw_graph_create: col must be in [0, nv) and strictly ascending per row; h finite and >= 0");
    }
    g->max_deg = (int64_t)host_chk[1];
    e = fw::launch_layout(g->row_ptr, g->col, g->h, g->nv, g->ne, g->edges, g->vrec, g->start_hi, nullptr);
    if (e == hipSuccess) e = hipMemset(g->scratch, 0, 4 * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        graph_free(g);
        return fail(FW_E_DEVICE, "fw_graph_create: %s", hipGetErrorString(e));
    }
    *out = g;
    return ok();
}

int fw_graph_destroy(fw_graph *g)
{
    graph_free(g);
    return ok();
}

int fw_graph_preprocess(fw_graph *g, void *stream)
{
    if (!g) return fail(FW_E_INVALID, "fw_graph_preprocess: null graph");
    HIP_TRY(hipSetDevice(g->device));
    HIP_TRY(fw::launch_preprocess(g->row_ptr, g->h, g->nv, g->vrec, (hipStream_t)stream));
    g->prepped = true;
    return ok();
}

int fw_graph_export_aux(const fw_graph *g, float *hmax, float *hsum)
{
    if (!g || !hmax || !hsum) return fail(FW_E_INVALID, "fw_graph_export_aux: null argument");
    if (!g->prepped) return fail(FW_E_STATE, "fw_graph_export_aux: graph not preprocessed");
    HIP_TRY(hipSetDevice(g->device));
    HIP_TRY(hipDeviceSynchronize());
    std::vector<uint4> rec((size_t)g->nv);
    if (g->nv > 0) HIP_TRY(hipMemcpy(rec.data(), g->vrec, sizeof(uint4) * rec.size(), hipMemcpyDeviceToHost));
    for (int64_t v = 0; v < g->nv; ++v) {
        uint32_t zb = rec[(size_t)v].z, wb = rec[(size_t)v].w;
        memcpy(&hmax[v], &zb, sizeof(float));
        memcpy(&hsum[v], &wb, sizeof(float));
    }
    return ok();
}

int fw_graph_info(const fw_graph *g, int64_t *nv, int64_t *ne, int64_t *max_deg)
{
    if (!g) return fail(FW_E_INVALID, "fw_graph_info: null graph");
    if (nv) *nv = g->nv;
    if (ne) *ne = g->ne;
    if (max_deg) *max_deg = g->max_deg;
    return ok();
}

int fw_logic_node2vec(float p, float q, int32_t weighted, fw_logic *out)
{
    if (!out) return fail(FW_E_INVALID, "fw_logic_node2vec: null output");
    if (!(p > 0.0f) || !(q > 0.0f) || isinf(p) || isinf(q))
        return fail(FW_E_INVALID, "fw_logic_node2vec: p and q must be finite and > 0");
    memset(out, 0, sizeof(*out));
    out->kind = FW_NODE2VEC;
    out->weighted = weighted ? 1 : 0;
    out->p = p;
    out->q = q;
    return ok();
}

int fw_logic_metapath(const uint8_t *schema, int32_t m, int32_t weighted, fw_logic *out)
{
    if (!out || !schema) return fail(FW_E_INVALID, "fw_logic_metapath: null argument");
    if (m < 1 || m > FW_MAX_SCHEMA) return fail(FW_E_INVALID, "fw_logic_metapath: 1 <= m <= %d", FW_MAX_SCHEMA);
    memset(out, 0, sizeof(*out));
    out->kind = FW_METAPATH;
    out->weighted = weighted ? 1 : 0;
    out->schema_len = m;
    memcpy(out->schema, schema, (size_t)m);
    return ok();
}

int fw_plan_default(fw_plan *out)
{
    if (!out) return fail(FW_E_INVALID, "fw_plan_default: null output");
    memset(out, 0, sizeof(*out));
    out->rho = 8.0f;
    out->d_lo = 0;
    out->rjs_cap = 1024;
    out->lanes = 64;
    out->lds_cap = fw::kDefaultLdsCap;
    out->grid = 0;
    return ok();
}

static int check_logic(const fw_graph *g, const fw_logic *lg)
{
    if (lg->kind == FW_NODE2VEC) {
        if (!(lg->p > 0.0f) || !(lg->q > 0.0f) || isinf(lg->p) || isinf(lg->q))
            return fail(FW_E_INVALID, "node2vec p and q must be finite and > 0");
    } else if (lg->kind == FW_METAPATH) {
        if (lg->schema_len < 1 || lg->schema_len > FW_MAX_SCHEMA)
            return fail(FW_E_INVALID, "metapath schema length must be in [1, %d]", FW_MAX_SCHEMA);
        if (!g->label) return fail(FW_E_INVALID, "metapath needs edge labels");
    } else {
        return fail(FW_E_INVALID, "unknown logic kind %d", lg->kind);
    }
    return FW_OK;
}

// Float constants of a launch, computed in float32 exactly as the definition states.
static void fill_args(const fw_graph *g, const fw_logic *lg, fw::WalkArgs &a)
{
    memset(&a, 0, sizeof(a));
    a.edges = g->edges;
    a.vrec = g->vrec;
    a.start_hi = g->start_hi;
    a.col = g->col;
    a.label = g->label;
    a.nv = g->nv;
    if (lg->kind == FW_NODE2VEC) {
        a.inv_p = 1.0f / lg->p;
        a.inv_q = 1.0f / lg->q;
        a.lo_w = fminf(1.0f, a.inv_q);
        a.hi_w = fmaxf(1.0f, a.inv_q);
        a.wmax0 = 1.0f;
        a.wavg0 = 1.0f;
        a.wmax1 = fmaxf(fmaxf(a.inv_p, 1.0f), a.inv_q);      // max over the three return values
        a.wavg1 = ((a.inv_p + 1.0f) + a.inv_q) / 3.0f;       // their mean (Section 4.2)
    } else {
        a.wmax0 = a.wmax1 = 1.0f;
        a.wavg0 = a.wavg1 = (1.0f + 0.0f) / 2.0f;
        a.schema_len = lg->schema_len;
        memcpy(a.schema, lg->schema, (size_t)lg->schema_len);
    }
    const bool weighted = lg->weighted && g->h;
    a.item_bytes = 4 + (weighted ? 4 : 0) + (lg->kind == FW_METAPATH ? 1 : 0);
}

int fw_walk(fw_graph *g, const fw_logic *lg, const fw_plan *pl, int32_t strategy, const int32_t *starts, int64_t n,
            int32_t L, uint64_t seed, int32_t *paths, int32_t *lengths, uint64_t *stats, void *stream)
{
    if (!g || !lg || !pl) return fail(FW_E_INVALID, "fw_walk: null graph, logic or plan");
    if (strategy < FW_AUTO || strategy > FW_RJS_ONLY) return fail(FW_E_INVALID, "fw_walk: bad strategy %d", strategy);
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(FW_E_INVALID, "fw_walk: n must be in [0, 2^31)");
    if (L < 0 || L >= (1 << 20)) return fail(FW_E_INVALID, "fw_walk: L must be in [0, 2^20)");
    if (n > 0 && (!starts || !paths || !lengths)) return fail(FW_E_INVALID, "fw_walk: null starts/paths/lengths");
    int rc = check_logic(g, lg);
    if (rc != FW_OK) return rc;
    if (pl->lanes != 64) return fail(FW_E_INVALID, "fw_walk: plan.lanes must be 64");
    if (pl->rjs_cap < 1) return fail(FW_E_INVALID, "fw_walk: plan.rjs_cap must be >= 1");
    if (!(pl->rho > 0.0f) || isinf(pl->rho)) return fail(FW_E_INVALID, "fw_walk: plan.rho must be finite and > 0");
    if (pl->d_lo < 0) return fail(FW_E_INVALID, "fw_walk: plan.d_lo must be >= 0");
    if (pl->lds_cap < 0 || pl->lds_cap > 16384) return fail(FW_E_INVALID, "fw_walk: plan.lds_cap in [0, 16384]");
    if (pl->grid < 0) return fail(FW_E_INVALID, "fw_walk: plan.grid must be >= 0");
    const bool weighted = lg->weighted && g->h;
    if (weighted && strategy != FW_RVS_ONLY && !g->prepped)
        return fail(FW_E_STATE, "fw_walk: call fw_graph_preprocess before a weighted eRJS/AUTO walk");
    if (n == 0) return ok();

    HIP_TRY(hipSetDevice(g->device));
    fw::WalkArgs a;
    fill_args(g, lg, a);
    a.starts = starts;
    a.n = n;
    a.L = L;
    a.paths = paths;
    a.lengths = lengths;
    a.stats = (unsigned long long *)stats;
    a.queue = g->scratch;
    a.err = (int *)(g->scratch + 1);
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    a.rho = pl->rho;
    a.d_lo = pl->d_lo;
    a.rjs_cap = pl->rjs_cap;
    a.strategy = strategy;
    a.lds_cap = pl->lds_cap;
    const int grid = pl->grid > 0 ? pl->grid : fw::walk_grid(lg->kind, weighted, a.lds_cap, n);
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(fw::launch_zero(g->scratch, 1, s));
    HIP_TRY(fw::launch_walk(a, lg->kind, weighted, grid, s));
    return ok();
}

int fw_graph_check(fw_graph *g, void *stream)
{
    if (!g) return fail(FW_E_INVALID, "fw_graph_check: null graph");
    HIP_TRY(hipSetDevice(g->device));
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    int flag = 0;
    HIP_TRY(hipMemcpy(&flag, g->scratch + 1, sizeof(int), hipMemcpyDeviceToHost));
    if (flag != 0) {
        HIP_TRY(hipMemset(g->scratch + 1, 0, sizeof(unsigned long long)));
        return fail(FW_E_INVALID, "fw_walk: a start vertex was outside [0, nv)");
    }
    return ok();
}

int fw_plan_autotune(fw_graph *g, const fw_logic *lg, fw_plan *out, void *stream)
{
    if (!g || !lg || !out) return fail(FW_E_INVALID, "fw_plan_autotune: null argument");
    int rc = check_logic(g, lg);
    if (rc != FW_OK) return rc;
    fw_plan_default(out);
    const bool weighted = lg->weighted && g->h;
    if (weighted && !g->prepped) return fail(FW_E_STATE, "fw_plan_autotune: graph not preprocessed");
    HIP_TRY(hipSetDevice(g->device));
    hipStream_t s = (hipStream_t)stream;

    // a fixed fraction of the non-isolated nodes, spread over the id range
    std::vector<int64_t> rp((size_t)g->nv + 1);
    HIP_TRY(hipMemcpy(rp.data(), g->row_ptr, sizeof(int64_t) * rp.size(), hipMemcpyDeviceToHost));
    std::vector<int32_t> nodes;
    int64_t nonempty = 0;
    for (int64_t v = 0; v < g->nv; ++v) nonempty += rp[v + 1] > rp[v];
    const int64_t want = std::min<int64_t>(nonempty, 16384);
    const int64_t stride = want > 0 ? std::max<int64_t>(1, nonempty / want) : 1;
    int64_t seen = 0;
    for (int64_t v = 0; v < g->nv && (int64_t)nodes.size() < want; ++v)
        if (rp[v + 1] > rp[v] && (seen++ % stride) == 0) nodes.push_back((int32_t)v);
    if (nodes.empty()) return ok();
    const int per_rvs = 256, per_rjs = 64;
    double e_rvs = 0, e_rjs = 0;
    for (int32_t v : nodes) {
        e_rvs += (double)std::min<int64_t>(rp[v + 1] - rp[v], per_rvs);
        e_rjs += per_rjs;
    }

    fw::WalkArgs a;
    fill_args(g, lg, a);
    a.key0 = 0x5eed;
    int32_t *d_nodes = nullptr;
    float *d_sink = nullptr;
    HIP_TRY(hipMalloc((void **)&d_nodes, sizeof(int32_t) * nodes.size()));
    HIP_TRY(hipMalloc((void **)&d_sink, sizeof(float)));
    HIP_TRY(hipMemcpy(d_nodes, nodes.data(), sizeof(int32_t) * nodes.size(), hipMemcpyHostToDevice));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best[2] = {1e30f, 1e30f};
    for (int style = 0; style < 2; ++style) {
        for (int rep = 0; rep < 4; ++rep) {
            HIP_TRY(hipEventRecord(e0, s));
            HIP_TRY(fw::launch_profile(a, lg->kind, weighted, style == 1, d_nodes, (int)nodes.size(),
                                       style == 1 ? per_rjs : per_rvs, d_sink, s));
            HIP_TRY(hipEventRecord(e1, s));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) best[style] = std::min(best[style], ms);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(d_nodes);
    (void)hipFree(d_sink);
    const double per_rvs_edge = best[0] / e_rvs, per_rjs_edge = best[1] / e_rjs;
    double rho = per_rjs_edge / per_rvs_edge;
    if (!(rho > 0.0)) rho = 8.0;
    out->rho = (float)std::min(1000.0, std::max(0.25, rho));
    return ok();
}

}  // extern "C"
