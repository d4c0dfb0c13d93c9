// C ABI of the sampler (include/flexiwalk.h): argument checks, device memory
// ownership, plan construction and kernel launches.  All sampling runs in
// fw_kernels.hip.
#include <float.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/flexiwalk.h"
#include "fw_device.h"
#include "fw_internal.h"
#include "fw_host.h"

namespace fw {
namespace host {

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

}  // namespace host
}  // namespace fw

using fw::host::check_logic;
using fw::host::check_bound;
using fw::host::check_plan;
using fw::host::fail;
using fw::host::fill_args;
using fw::host::fill_query;
using fw::host::ok;
using fw::host::plan_args;

static void graph_free(fw_graph *g)
{
    if (!g) return;
    (void)hipFree(g->row_ptr);
    (void)hipFree(g->col);
    (void)hipFree(g->h);
    (void)hipFree(g->label);
    (void)hipFree(g->edges);
    (void)hipFree(g->erec8);
    (void)hipFree(g->vrec);
    (void)hipFree(g->start_hi);
    (void)hipFree(g->scratch);
    (void)hipFree(g->mtab);
    (void)hipFree(g->prop);
    (void)hipFree(g->lrow);
    (void)hipFree(g->lprop);
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

// device memory freed at scope exit
struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { (void)hipFree(p); }
};

extern "C" {

const char *fw_last_error(void) { return fw::host::g_err.c_str(); }

int fw_graph_create(const fw_csr *in, fw_graph **out)
{
    if (!in || !out) return fail(FW_E_INVALID, "fw_graph_create: null argument");
    if (in->nv < 0 || in->ne < 0) return fail(FW_E_INVALID, "fw_graph_create: negative size");
    // vertex ids, degrees and search brackets are int32 on the device
    if (in->nv >= ((int64_t)1 << 30)) return fail(FW_E_INVALID, "fw_graph_create: nv must be < 2^30");
    if (!in->row_ptr || (in->ne > 0 && !in->col))
        return fail(FW_E_INVALID, "fw_graph_create: row_ptr/col missing");
    if (in->h8 && in->h) return fail(FW_E_INVALID, "fw_graph_create: give h or h8, not both");
    if (in->h8 && !(in->h_scale > 0.0f && in->h_scale <= FLT_MAX))
        return fail(FW_E_INVALID, "fw_graph_create: h_scale must be finite and > 0 with h8");

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
    // 8-bit weights: the dequantised h serves preprocessing, validation and the index and
    // proposal builds; the walk reads 4-byte records {col, code} when vertex ids fit 24 bits
    DevBuf codes;
    if (in->h8) {
        g->q8 = true;
        g->h_scale = in->h_scale;
        if ((rc = dev_copy((uint8_t **)&codes.p, in->h8, in->ne, in->on_device)) != FW_OK) {
            graph_free(g);
            return rc;
        }
        if (hipMalloc((void **)&g->h, sizeof(float) * (size_t)(g->ne > 0 ? g->ne : 1)) != hipSuccess) {
            graph_free(g);
            return fail(FW_E_NOMEM, "fw_graph_create: hipMalloc failed");
        }
        const hipError_t e = fw::launch_dequantize((const uint8_t *)codes.p, g->h_scale, g->ne, g->h, nullptr);
        if (e != hipSuccess) {
            graph_free(g);
            return fail(FW_E_DEVICE, "fw_graph_create: %s", hipGetErrorString(e));
        }
    }
    const bool packed = g->q8 && g->nv <= ((int64_t)1 << 24);
    const bool wide = g->ne >= ((int64_t)1 << 32);
    if ((packed && hipMalloc((void **)&g->erec8, sizeof(uint32_t) * (size_t)(g->ne > 0 ? g->ne : 1)) != hipSuccess) ||
        (!packed && hipMalloc((void **)&g->edges, sizeof(uint2) * (size_t)(g->ne > 0 ? g->ne : 1)) != hipSuccess) ||
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
    // symmetry decides whether the split eRJS bound may be used; not an error
    e = fw::launch_check_symmetry(g->row_ptr, g->col, g->h, g->nv, (int *)chk, nullptr);
    if (e == hipSuccess) e = hipMemcpy(host_chk, chk, sizeof(host_chk), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        graph_free(g);
        return fail(FW_E_DEVICE, "fw_graph_create: %s", hipGetErrorString(e));
    }
    g->symmetric = (host_chk[0] & 16u) == 0;
    e = fw::launch_layout(g->row_ptr, g->col, g->h, g->nv, g->ne, g->edges, g->vrec, g->start_hi, nullptr);
    if (e == hipSuccess && packed) e = fw::launch_pack8(g->col, (const uint8_t *)codes.p, g->ne, g->erec8, nullptr);
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

int fw_graph_build_index(fw_graph *g, void *stream)
{
    if (!g) return fail(FW_E_INVALID, "fw_graph_build_index: null graph");
    if (g->mtab) return ok();
    HIP_TRY(hipSetDevice(g->device));
    // power-of-two count of 128-byte buckets with at least 16 slots per 8 keys (load <= 1/2)
    uint64_t buckets = 1;
    while (buckets * 8 < 2 * (uint64_t)g->ne) buckets <<= 1;
    unsigned long long *tab = nullptr;
    if (hipMalloc((void **)&tab, buckets * 128) != hipSuccess)
        return fail(FW_E_NOMEM, "fw_graph_build_index: hipMalloc of %llu bytes failed",
                    (unsigned long long)(buckets * 128));
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemsetAsync(tab, 0xFF, buckets * 128, s);  // every key kEmptyKey
    if (e == hipSuccess) e = fw::launch_build_index(g->row_ptr, g->col, g->h, g->nv, tab, buckets - 1, s);
    if (e != hipSuccess) {
        (void)hipFree(tab);
        return fail(FW_E_DEVICE, "fw_graph_build_index: %s", hipGetErrorString(e));
    }
    g->mtab = tab;
    g->mtab_mask = buckets - 1;
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

int fw_graph_export_alias(const fw_graph *g, uint32_t *thr, int32_t *alias)
{
    if (!g || (g->ne > 0 && (!thr || !alias))) return fail(FW_E_INVALID, "fw_graph_export_alias: null argument");
    if (!g->prop) return fail(FW_E_STATE, "fw_graph_export_alias: no proposal records (fw_graph_build_alias)");
    if (g->ne == 0) return ok();
    HIP_TRY(hipSetDevice(g->device));
    HIP_TRY(hipDeviceSynchronize());
    // gathered on the device from the second uint4 of each record, then copied whole
    DevBuf dt, da;
    HIP_TRY(hipMalloc(&dt.p, sizeof(uint32_t) * (size_t)g->ne));
    HIP_TRY(hipMalloc(&da.p, sizeof(int32_t) * (size_t)g->ne));
    HIP_TRY(fw::launch_export_alias(g->prop, g->ne, (uint32_t *)dt.p, (int32_t *)da.p, nullptr));
    HIP_TRY(hipMemcpy(thr, dt.p, sizeof(uint32_t) * (size_t)g->ne, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(alias, da.p, sizeof(int32_t) * (size_t)g->ne, hipMemcpyDeviceToHost));
    return ok();
}

int fw_graph_info(const fw_graph *g, int64_t *nv, int64_t *ne, int64_t *max_deg, int32_t *symmetric)
{
    if (!g) return fail(FW_E_INVALID, "fw_graph_info: null graph");
    if (nv) *nv = g->nv;
    if (ne) *ne = g->ne;
    if (max_deg) *max_deg = g->max_deg;
    if (symmetric) *symmetric = g->symmetric ? 1 : 0;
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

int fw_logic_second_pr(float gamma, int32_t weighted, fw_logic *out)
{
    if (!out) return fail(FW_E_INVALID, "fw_logic_second_pr: null output");
    if (!(gamma >= 0.0f && gamma <= 1.0f)) return fail(FW_E_INVALID, "second-order PageRank gamma must be in [0, 1]");
    memset(out, 0, sizeof(*out));
    out->kind = FW_SECOND_PR;
    out->weighted = weighted ? 1 : 0;
    out->gamma = gamma;
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
    out->bound = 0;
    out->hub_deg = 0;
    out->hub_lanes = 64;
    out->rvs_share = 0;
    return ok();
}

}  // extern "C"

int fw::host::check_logic(const fw_graph *g, const fw_logic *lg)
{
    if (lg->kind == FW_NODE2VEC) {
        if (!(lg->p > 0.0f) || !(lg->q > 0.0f) || isinf(lg->p) || isinf(lg->q))
            return fail(FW_E_INVALID, "node2vec p and q must be finite and > 0");
    } else if (lg->kind == FW_METAPATH) {
        if (lg->schema_len < 1 || lg->schema_len > FW_MAX_SCHEMA)
            return fail(FW_E_INVALID, "metapath schema length must be in [1, %d]", FW_MAX_SCHEMA);
        if (!g->label) return fail(FW_E_INVALID, "metapath needs edge labels");
    } else if (lg->kind == FW_SECOND_PR) {
        if (!(lg->gamma >= 0.0f && lg->gamma <= 1.0f))
            return fail(FW_E_INVALID, "second-order PageRank gamma must be in [0, 1]");
    } else {
        return fail(FW_E_INVALID, "unknown logic kind %d", lg->kind);
    }
    return FW_OK;
}

// Per-query float constants, computed in float32 exactly as the definition states.
void fw::host::fill_query(const fw_logic *lg, fw::QueryDev &q)
{
    memset(&q, 0, sizeof(q));
    if (lg->kind == FW_NODE2VEC) {
        q.inv_p = 1.0f / lg->p;
        q.inv_q = 1.0f / lg->q;
        q.lo_w = fminf(1.0f, q.inv_q);
        q.hi_w = fmaxf(1.0f, q.inv_q);
        q.wmax0 = 1.0f;
        q.wavg0 = 1.0f;
        q.wmax1 = fmaxf(fmaxf(q.inv_p, 1.0f), q.inv_q);      // max over the three return values
        q.wavg1 = ((q.inv_p + 1.0f) + q.inv_q) / 3.0f;       // their mean (Section 4.2)
    } else if (lg->kind == FW_SECOND_PR) {
        // step 0 uses w = 1; later steps take max and mean of the two branches of
        // Eq. (2ndpr), which depend on the step's degrees (computed in the kernel)
        q.gamma = lg->gamma;
        q.omg = 1.0f - lg->gamma;
        q.wmax0 = q.wavg0 = 1.0f;
        q.wmax1 = q.wavg1 = 1.0f;
    } else {
        q.wmax0 = q.wmax1 = 1.0f;
        q.wavg0 = q.wavg1 = (1.0f + 0.0f) / 2.0f;
        q.schema_len = lg->schema_len;
        memcpy(q.schema, lg->schema, (size_t)lg->schema_len);
    }
}

void fw::host::fill_args(const fw_graph *g, const fw_logic *lg, fw::WalkArgs &a)
{
    memset(&a, 0, sizeof(a));
    a.edges = g->edges;
    a.erec8 = g->erec8;
    a.h_scale = g->h_scale;
    a.vrec = g->vrec;
    a.start_hi = g->start_hi;
    a.col = g->col;
    a.label = g->label;
    a.nv = g->nv;
    a.mtab = (const uint4 *)g->mtab;
    a.mtab_mask = g->mtab_mask;
    a.prop = g->prop;
    a.lrow = g->lrow;
    a.lprop = g->lprop;
    a.nlab = g->nlab;
    fill_query(lg, a.q0);
    const bool weighted = lg->weighted && g->h;
    a.item_bytes = 4 + (weighted ? (g->q8 ? 1 : 4) : 0) + (lg->kind == FW_METAPATH ? 1 : 0);
}

int fw::host::check_plan(const fw_plan *pl)
{
    if (pl->lanes != 64) return fail(FW_E_INVALID, "plan.lanes must be 64");
    if (pl->rjs_cap < 1) return fail(FW_E_INVALID, "plan.rjs_cap must be >= 1");
    if (!(pl->rho > 0.0f) || isinf(pl->rho)) return fail(FW_E_INVALID, "plan.rho must be finite and > 0");
    if (pl->d_lo < 0) return fail(FW_E_INVALID, "plan.d_lo must be >= 0");
    if (pl->lds_cap < 0 || pl->lds_cap > fw::kMaxLdsCap)
        return fail(FW_E_INVALID, "plan.lds_cap in [0, %d]", fw::kMaxLdsCap);
    if (pl->grid < 0) return fail(FW_E_INVALID, "plan.grid must be >= 0");
    if (pl->bound < 0 || pl->bound > 2) return fail(FW_E_INVALID, "plan.bound must be 0, 1 or 2");
    if (pl->proposal < 0 || pl->proposal > 2) return fail(FW_E_INVALID, "plan.proposal must be 0, 1 or 2");
    if (pl->hub_deg < 0) return fail(FW_E_INVALID, "plan.hub_deg must be >= 0");
    if (pl->hub_lanes != 64 && pl->hub_lanes != 128 && pl->hub_lanes != 256)
        return fail(FW_E_INVALID, "plan.hub_lanes must be 64, 128 or 256");
    if (pl->rvs_share != 0 && pl->rvs_share != 1) return fail(FW_E_INVALID, "plan.rvs_share must be 0 or 1");
    return FW_OK;
}

int fw::host::check_bound(const fw_graph *g, const fw_plan *pl, const fw_logic *lg)
{
    const bool lab = pl->proposal == 2 && lg->kind == FW_METAPATH;
    if (pl->proposal >= 1 && !lab && lg->weighted && g->h && !g->prop)
        return fail(FW_E_STATE, "plan.proposal = %d needs fw_graph_build_alias first", (int)pl->proposal);
    if (lab && !g->lprop)
        return fail(FW_E_STATE, "plan.proposal = 2 with a MetaPath logic needs fw_graph_build_label_alias first");
    if (pl->bound >= 1 && lg->kind == FW_NODE2VEC && !g->symmetric)
        return fail(FW_E_INVALID, "plan.bound = %d needs every edge's reverse with the same h (fw_graph_info)",
                    (int)pl->bound);
    return FW_OK;
}

void fw::host::plan_args(const fw_plan *pl, int32_t strategy, fw::WalkArgs &a)
{
    a.rho = pl->rho;
    a.d_lo = pl->d_lo;
    a.rjs_cap = pl->rjs_cap;
    a.strategy = strategy;
    a.lds_cap = pl->lds_cap;
    a.bound = pl->bound;
    a.proposal = pl->proposal;
    a.hub_deg = pl->hub_deg;
    a.hub_v = pl->hub_lanes / 64;
    a.rvs_share = pl->rvs_share;
}

extern "C" {

int fw_walk(fw_graph *g, const fw_logic *lg, const fw_plan *pl, int32_t strategy, const int32_t *starts, int64_t n,
            int32_t L, uint64_t seed, int32_t *paths, int32_t *lengths, uint64_t *stats, void *stream)
{
    if (!g || !lg || !pl) return fail(FW_E_INVALID, "fw_walk: null graph, logic or plan");
    if (!fw::valid_strategy(strategy)) return fail(FW_E_INVALID, "fw_walk: bad strategy %d", strategy);
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(FW_E_INVALID, "fw_walk: n must be in [0, 2^31)");
    if (L < 0 || L >= (1 << 20)) return fail(FW_E_INVALID, "fw_walk: L must be in [0, 2^20)");
    if (n > 0 && (!starts || !paths || !lengths)) return fail(FW_E_INVALID, "fw_walk: null starts/paths/lengths");
    int rc = check_logic(g, lg);
    if (rc != FW_OK) return rc;
    if ((rc = check_plan(pl)) != FW_OK) return rc;
    if ((rc = check_bound(g, pl, lg)) != FW_OK) return rc;
    const bool weighted = lg->weighted && g->h;
    if (weighted && strategy != FW_RVS_ONLY && !g->prepped)
        return fail(FW_E_STATE, "fw_walk: call fw_graph_preprocess before a weighted eRJS/AUTO walk");
    if (n == 0) return ok();

    HIP_TRY(hipSetDevice(g->device));
    fw::WalkArgs a;
    fill_args(g, lg, a);
    plan_args(pl, strategy, a);
    a.n = n;
    a.stats = (unsigned long long *)stats;
    a.queue = g->scratch;
    a.err = (int *)(g->scratch + 1);
    a.q0.first = 0;
    a.q0.n = n;
    a.q0.starts = starts;
    a.q0.paths = paths;
    a.q0.lengths = lengths;
    a.q0.L = L;
    a.q0.key0 = (uint32_t)seed;
    a.q0.key1 = (uint32_t)(seed >> 32);
    a.nq = 1;
    const int grid =
        pl->grid > 0 ? pl->grid : fw::walk_grid(lg->kind, weighted, false, a.lds_cap, n, strategy == FW_RVS_ONLY);
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(fw::launch_zero(g->scratch, 1, s));
    HIP_TRY(fw::launch_walk(a, lg->kind, weighted, false, grid, s));
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

// Device buffer released on scope exit.
struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

int fw_graph_build_alias(fw_graph *g, void *stream)
{
    if (!g) return fail(FW_E_INVALID, "fw_graph_build_alias: null graph");
    if (g->prop) return ok();
    HIP_TRY(hipSetDevice(g->device));
    // the records carry the candidates' vertex records, h_MAX and h_SUM included
    if (!g->prepped) {
        const int rc = fw_graph_preprocess(g, stream);
        if (rc != FW_OK) return rc;
    }
    const size_t ne = (size_t)(g->ne > 0 ? g->ne : 1);
    const size_t rec = 16 * (size_t)fw::kPropU4;
    uint4 *prop = nullptr;
    if (hipMalloc((void **)&prop, rec * ne) != hipSuccess)
        return fail(FW_E_NOMEM, "fw_graph_build_alias: hipMalloc of %zu bytes failed", rec * ne);
    DevBuf val, idx, rowinfo, hubs, nhub;
    const size_t nv = (size_t)(g->nv > 0 ? g->nv : 1);
    if (hipMalloc(&val.p, 16 * ne) != hipSuccess || hipMalloc(&idx.p, 4 * ne) != hipSuccess ||
        hipMalloc(&rowinfo.p, 16 * nv) != hipSuccess || hipMalloc(&hubs.p, 4 * nv) != hipSuccess ||
        hipMalloc(&nhub.p, sizeof(int)) != hipSuccess) {
        (void)hipFree(prop);
        return fail(FW_E_NOMEM, "fw_graph_build_alias: scratch of %zu bytes failed", 20 * ne + 20 * nv);
    }
    hipStream_t s = (hipStream_t)stream;
    // every record is written by the build; zeroed first so that none can ever hold an
    // out-of-range vertex
    hipError_t e = hipMemsetAsync(prop, 0, rec * ne, s);
    if (e == hipSuccess)
        e = fw::launch_build_alias(g->row_ptr, g->col, g->h, g->label, g->nv, g->vrec, nullptr, (uint4 *)val.p,
                                   (int32_t *)idx.p, (ulonglong2 *)rowinfo.p, (int32_t *)hubs.p, (int *)nhub.p, prop,
                                   s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(prop);
        return fail(FW_E_DEVICE, "fw_graph_build_alias: %s", hipGetErrorString(e));
    }
    g->prop = prop;
    return ok();
}

int fw_graph_build_label_alias(fw_graph *g, void *stream)
{
    if (!g) return fail(FW_E_INVALID, "fw_graph_build_label_alias: null graph");
    if (!g->label) return fail(FW_E_STATE, "fw_graph_build_label_alias: the graph has no edge labels");
    if (g->lprop) return ok();
    HIP_TRY(hipSetDevice(g->device));
    // the records carry the candidates' vertex records, h_MAX and h_SUM included
    if (!g->prepped) {
        const int rc = fw_graph_preprocess(g, stream);
        if (rc != FW_OK) return rc;
    }
    hipStream_t s = (hipStream_t)stream;
    int mx = 0;
    {
        DevBuf d;
        HIP_TRY(hipMalloc(&d.p, sizeof(int)));
        HIP_TRY(hipMemsetAsync(d.p, 0, sizeof(int), s));
        HIP_TRY(fw::launch_label_max(g->label, g->ne, (int *)d.p, s));
        HIP_TRY(hipMemcpyAsync(&mx, d.p, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    const int nlab = mx + 1;
    if (nlab > fw::kMaxLabels)
        return fail(FW_E_INVALID, "fw_graph_build_label_alias: label %d; label groups take labels below %d", mx,
                    fw::kMaxLabels);
    const size_t ne = (size_t)(g->ne > 0 ? g->ne : 1);
    const size_t ng = (size_t)g->nv * (size_t)nlab;  // groups
    const size_t rec = 16 * (size_t)fw::kPropU4;
    int64_t *lrow = nullptr;
    uint4 *lprop = nullptr;
    if (hipMalloc((void **)&lrow, sizeof(int64_t) * (ng + 1)) != hipSuccess) {
        return fail(FW_E_NOMEM, "fw_graph_build_label_alias: hipMalloc of %zu bytes failed", 8 * (ng + 1));
    }
    if (hipMalloc((void **)&lprop, rec * ne) != hipSuccess) {
        (void)hipFree(lrow);
        return fail(FW_E_NOMEM, "fw_graph_build_label_alias: hipMalloc of %zu bytes failed", rec * ne);
    }
    DevBuf gmax, vcol, vh, vlab, val, idx, rowinfo, hubs, nhub;
    const size_t ngr = ng > 0 ? ng : 1;
    if (hipMalloc(&gmax.p, 4 * ngr) != hipSuccess || hipMalloc(&vcol.p, 4 * ne) != hipSuccess ||
        (g->h && hipMalloc(&vh.p, 4 * ne) != hipSuccess) || hipMalloc(&vlab.p, ne) != hipSuccess ||
        hipMalloc(&val.p, 16 * ne) != hipSuccess || hipMalloc(&idx.p, 4 * ne) != hipSuccess ||
        hipMalloc(&rowinfo.p, 16 * ngr) != hipSuccess || hipMalloc(&hubs.p, 4 * ngr) != hipSuccess ||
        hipMalloc(&nhub.p, sizeof(int)) != hipSuccess) {
        (void)hipFree(lrow);
        (void)hipFree(lprop);
        return fail(FW_E_NOMEM, "fw_graph_build_label_alias: scratch of %zu bytes failed", 29 * ne + 24 * ngr);
    }
    const int64_t total = g->ne;
    // every record is written by the build; zeroed first so that none can ever hold an
    // out-of-range vertex
    hipError_t e = hipMemsetAsync(lprop, 0, rec * ne, s);
    if (e == hipSuccess)
        e = fw::launch_label_groups(g->row_ptr, g->col, g->h, g->label, g->nv, nlab, lrow, (float *)gmax.p,
                                    (int32_t *)vcol.p, (float *)vh.p, (uint8_t *)vlab.p, s);
    if (e == hipSuccess) e = hipMemcpyAsync(lrow + ng, &total, sizeof(int64_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = fw::launch_build_alias(lrow, (const int32_t *)vcol.p, (const float *)vh.p, (const uint8_t *)vlab.p,
                                   (int64_t)ng, g->vrec, (const float *)gmax.p, (uint4 *)val.p, (int32_t *)idx.p,
                                   (ulonglong2 *)rowinfo.p, (int32_t *)hubs.p, (int *)nhub.p, lprop, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(lrow);
        (void)hipFree(lprop);
        return fail(FW_E_DEVICE, "fw_graph_build_label_alias: %s", hipGetErrorString(e));
    }
    g->lrow = lrow;
    g->lprop = lprop;
    g->nlab = nlab;
    return ok();
}

int fw_calibrate_random_reads(int64_t bytes, double *reads_per_s, void *stream)
{
    if (!reads_per_s) return fail(FW_E_INVALID, "fw_calibrate_random_reads: null output");
    if (bytes < (1 << 20) || (bytes & (bytes - 1)) != 0)
        return fail(FW_E_INVALID, "fw_calibrate_random_reads: bytes must be a power of two >= 1 MiB");
    hipStream_t s = (hipStream_t)stream;
    DevBuf arr, sink;
    HIP_TRY(hipMalloc(&arr.p, (size_t)bytes));
    HIP_TRY(hipMalloc(&sink.p, sizeof(unsigned)));
    HIP_TRY(hipMemsetAsync(arr.p, 1, (size_t)bytes, s));
    const uint64_t mask = (uint64_t)bytes / 8 - 1;
    const int blocks = 4096, rounds = 64;
    Events ev;
    HIP_TRY(hipEventCreate(&ev.a));
    HIP_TRY(hipEventCreate(&ev.b));
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {  // the first launch warms up; the fastest counts
        HIP_TRY(hipEventRecord(ev.a, s));
        HIP_TRY(fw::launch_random_reads((const uint2 *)arr.p, mask, blocks, rounds, (unsigned *)sink.p, s));
        HIP_TRY(hipEventRecord(ev.b, s));
        HIP_TRY(hipEventSynchronize(ev.b));
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
        if (rep > 0) best = std::min(best, ms);
    }
    *reads_per_s = (double)blocks * fw::kBlock * rounds * 4 / (best / 1e3);
    return ok();
}

int fw_plan_profile(fw_graph *g, const fw_logic *lg, fw_plan *out, void *stream)
{
    if (!g || !lg || !out) return fail(FW_E_INVALID, "fw_plan_profile: null argument");
    int rc = check_logic(g, lg);
    if (rc != FW_OK) return rc;
    fw_plan_default(out);
    const bool weighted = lg->weighted && g->h;
    if (weighted && !g->prepped) return fail(FW_E_STATE, "fw_plan_profile: graph not preprocessed");
    HIP_TRY(hipSetDevice(g->device));
    hipStream_t s = (hipStream_t)stream;

    // up to 16384 non-isolated nodes spread over the id range: 32768 evenly spaced
    // candidates (every vertex of a smaller graph), read on the device, keeping the
    // non-isolated ones in id order
    const int64_t ncand = std::min<int64_t>(g->nv, 32768);
    if (ncand == 0) return ok();
    const int64_t stride = std::max<int64_t>(1, g->nv / std::max<int64_t>(1, ncand));
    std::vector<int2> cand((size_t)ncand);
    {
        DevBuf d_cand;
        HIP_TRY(hipMalloc(&d_cand.p, sizeof(int2) * cand.size()));
        HIP_TRY(fw::launch_profile_pick(g->row_ptr, stride, (int)ncand, (int2 *)d_cand.p, s));
        HIP_TRY(hipMemcpyAsync(cand.data(), d_cand.p, sizeof(int2) * cand.size(), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    std::vector<int32_t> nodes;
    const int per_rvs = 256, per_rjs = 64;
    double e_rvs = 0, e_rjs = 0;
    for (const int2 &c : cand) {
        if (c.y <= 0 || nodes.size() >= 16384) continue;
        nodes.push_back(c.x);
        e_rvs += (double)std::min<int32_t>(c.y, per_rvs);
        e_rjs += per_rjs;
    }
    if (nodes.empty()) return ok();

    fw::WalkArgs a;
    fill_args(g, lg, a);
    a.q0.key0 = 0x5eed;
    DevBuf d_nodes, d_sink;
    HIP_TRY(hipMalloc(&d_nodes.p, sizeof(int32_t) * nodes.size()));
    HIP_TRY(hipMalloc(&d_sink.p, sizeof(float)));
    HIP_TRY(hipMemcpy(d_nodes.p, nodes.data(), sizeof(int32_t) * nodes.size(), hipMemcpyHostToDevice));
    Events ev;
    HIP_TRY(hipEventCreate(&ev.a));
    HIP_TRY(hipEventCreate(&ev.b));
    float best[2] = {1e30f, 1e30f};
    for (int style = 0; style < 2; ++style) {
        for (int rep = 0; rep < 4; ++rep) {
            HIP_TRY(hipEventRecord(ev.a, s));
            HIP_TRY(fw::launch_profile(a, lg->kind, weighted, style == 1, (const int32_t *)d_nodes.p,
                                       (int)nodes.size(), style == 1 ? per_rjs : per_rvs, (float *)d_sink.p, s));
            HIP_TRY(hipEventRecord(ev.b, s));
            HIP_TRY(hipEventSynchronize(ev.b));
            float ms = 0;
            HIP_TRY(hipEventElapsedTime(&ms, ev.a, ev.b));
            if (rep > 0) best[style] = std::min(best[style], ms);
        }
    }
    const double per_rvs_edge = best[0] / e_rvs, per_rjs_edge = best[1] / e_rjs;
    double rho = per_rjs_edge / per_rvs_edge;
    if (!(rho > 0.0)) rho = 8.0;
    out->rho = (float)std::min(1000.0, std::max(0.25, rho));
    return ok();
}

int fw_plan_autotune(fw_graph *g, const fw_logic *lg, fw_plan *out, void *stream)
{
    return fw_plan_autotune_mix(g, lg, 1, out, stream);
}

int fw_plan_autotune_mix(fw_graph *g, const fw_logic *logics, int32_t n_logics, fw_plan *out, void *stream)
{
    if (!g || !logics || !out || n_logics < 1 || n_logics > 64)
        return fail(FW_E_INVALID, "fw_plan_autotune_mix: null argument or n_logics outside 1..64");
    int rc = fw_plan_profile(g, &logics[0], out, stream);
    if (rc != FW_OK) return rc;
    for (int32_t i = 1; i < n_logics; ++i)
        if ((rc = check_logic(g, &logics[i])) != FW_OK) return rc;
    if (g->nv == 0 || g->ne == 0) return ok();
    hipStream_t s = (hipStream_t)stream;

    // sample walks: seeded walkers spread over all vertices, enough to keep the device busy
    // for milliseconds per candidate (shorter runs time the launch and the tail), long
    // enough for the walk's degree bias to set in; with several logics each runs at least
    // 2^18 walkers (shorter runs time noise) and a candidate's time is the sum over the logics
    const int64_t n = std::min<int64_t>(g->nv, std::max<int64_t>(1 << 18, (1 << 20) / n_logics));
    const int32_t L = 16;
    // a mix that one batch can hold (one kind and weighting) is timed as such a batch, one
    // query per logic, so that the batched kernel a batch or a server runs is what is
    // measured; otherwise each logic is timed in fw_walk launches of its own
    bool batched = n_logics > 1;
    for (int32_t i = 1; i < n_logics; ++i)
        batched = batched && logics[i].kind == logics[0].kind &&
                  (logics[i].weighted != 0) == (logics[0].weighted != 0);
    const int64_t nq = batched ? n_logics : 1;
    std::vector<int32_t> starts((size_t)n);
    uint64_t x = 0x9E3779B97F4A7C15ull;
    for (int64_t i = 0; i < n; ++i) {
        x ^= x << 13;
        x ^= x >> 7;
        x ^= x << 17;
        starts[(size_t)i] = (int32_t)(x % (uint64_t)g->nv);
    }
    DevBuf d_starts, d_paths, d_len;
    HIP_TRY(hipMalloc(&d_starts.p, sizeof(int32_t) * (size_t)n));
    HIP_TRY(hipMalloc(&d_paths.p, sizeof(int32_t) * (size_t)(nq * n * (L + 1))));
    HIP_TRY(hipMalloc(&d_len.p, sizeof(int32_t) * (size_t)(nq * n)));
    HIP_TRY(hipMemcpy(d_starts.p, starts.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice));
    Events ev;
    HIP_TRY(hipEventCreate(&ev.a));
    HIP_TRY(hipEventCreate(&ev.b));
    std::vector<fw_query> qs((size_t)nq);
    for (int64_t i = 0; i < nq; ++i) {
        qs[(size_t)i].logic = logics[i];
        qs[(size_t)i].n = n;
        qs[(size_t)i].L = L;
        qs[(size_t)i].seed = 7 + (uint64_t)i;
        qs[(size_t)i].start_off = 0;  // every query starts from the same sample
        qs[(size_t)i].out_off = i * n * (L + 1);
        qs[(size_t)i].len_off = i * n;
    }
    auto time_batch = [&](const fw_plan &p, float *ms) -> int {
        fw_batch *b = nullptr;
        int r = fw_batch_create(g, qs.data(), nq, &p, FW_AUTO, (const int32_t *)d_starts.p, n, (int32_t *)d_paths.p,
                                nq * n * (L + 1), (int32_t *)d_len.p, nq * n, &b);
        if (r != FW_OK) return r;
        float best = 1e30f;
        for (int rep = 0; rep < 2 && r == FW_OK; ++rep) {
            float t = 0;
            if (hipEventRecord(ev.a, s) != hipSuccess || (r = fw_batch_launch(b, nullptr, stream)) != FW_OK ||
                hipEventRecord(ev.b, s) != hipSuccess || hipEventSynchronize(ev.b) != hipSuccess ||
                hipEventElapsedTime(&t, ev.a, ev.b) != hipSuccess) {
                if (r == FW_OK) r = fail(FW_E_DEVICE, "fw_plan_autotune_mix: timing a batch failed");
                break;
            }
            best = std::min(best, t);
        }
        (void)hipStreamSynchronize(s);
        (void)fw_batch_destroy(b);
        *ms = best;
        return r;
    };
    auto time_plan = [&](const fw_plan &p, float *ms) -> int {
        if (batched) return time_batch(p, ms);
        float total = 0;
        for (int32_t i = 0; i < n_logics; ++i) {
            float best = 1e30f;
            for (int rep = 0; rep < 2; ++rep) {
                HIP_TRY(hipEventRecord(ev.a, s));
                int r = fw_walk(g, &logics[i], &p, FW_AUTO, (const int32_t *)d_starts.p, n, L, 7 + (uint64_t)i,
                                (int32_t *)d_paths.p, (int32_t *)d_len.p, nullptr, stream);
                if (r != FW_OK) return r;
                HIP_TRY(hipEventRecord(ev.b, s));
                HIP_TRY(hipEventSynchronize(ev.b));
                float t = 0;
                HIP_TRY(hipEventElapsedTime(&t, ev.a, ev.b));
                best = std::min(best, t);
            }
            total += best;
        }
        *ms = total;
        return FW_OK;
    };
    // bounds every logic accepts: 0 always; the split bound (1) when a Node2Vec logic is
    // present and the graph is symmetric; the member board (2) then, or for second-order
    // PageRank when no Node2Vec logic needs a symmetric graph that is missing
    bool any_n2v = false, any_pr = false, any_weighted = false;
    for (int32_t i = 0; i < n_logics; ++i) {
        any_n2v = any_n2v || logics[i].kind == FW_NODE2VEC;
        any_pr = any_pr || logics[i].kind == FW_SECOND_PR;
        any_weighted = any_weighted || logics[i].weighted;
    }
    int32_t bounds[3] = {0, 0, 0};
    int nbound = 1;
    if (any_n2v && g->symmetric) bounds[nbound++] = 1;
    if ((any_n2v && g->symmetric) || (any_pr && !any_n2v)) bounds[nbound++] = 2;
    // proposals: uniform; h-proportional for a weighted logic once the records exist;
    // label-conditioned for MetaPath once the label groups exist (the mix's other logics
    // then take h-proportional proposals, whose records a weighted one needs)
    bool any_mp = false, any_w_other = false;
    for (int32_t i = 0; i < n_logics; ++i) {
        any_mp = any_mp || logics[i].kind == FW_METAPATH;
        any_w_other = any_w_other || (logics[i].kind != FW_METAPATH && logics[i].weighted);
    }
    int32_t props[3] = {0, 0, 0};
    int nprop = 1;
    if (any_weighted && g->h && g->prop) props[nprop++] = 1;
    if (any_mp && g->lprop && (!any_w_other || !g->h || g->prop)) props[nprop++] = 2;
    // cost-model constant around the profiled value for each bound and proposal, then the
    // degree gate, the LDS budget for N(prev), the eRJS trial cap and the persistent grid
    fw_plan bestp = *out;
    float bestt = 1e30f;
    const float rho0 = out->rho;
    const float scales[] = {0.0625f, 0.25f, 0.5f, 1.0f, 2.0f, 4.0f};
    for (int ip = 0; ip < nprop; ++ip) {
        for (int ib = 0; ib < nbound; ++ib) {
            for (float sc : scales) {
                fw_plan p = *out;
                p.rho = std::max(1e-3f, rho0 * sc);
                p.bound = bounds[ib];
                p.proposal = props[ip];
                float t;
                if ((rc = time_plan(p, &t)) != FW_OK) return rc;
                if (t < bestt) bestt = t, bestp = p;
            }
        }
    }
    for (int32_t d : {8, 32, 128}) {
        fw_plan p = bestp;
        p.d_lo = d;
        float t;
        if ((rc = time_plan(p, &t)) != FW_OK) return rc;
        if (t < bestt) bestt = t, bestp = p;
    }
    for (int32_t cap : {256, 1024, 2048, 4096}) {  // around the default of 512
        fw_plan p = bestp;
        p.lds_cap = cap;
        float t;
        if ((rc = time_plan(p, &t)) != FW_OK) return rc;
        if (t < bestt) bestt = t, bestp = p;
    }
    // the trial cap K: a step past it falls back to eRVS (an exact sample either way), so a
    // small cap bounds the time a lane spends where the bound is loose
    for (int32_t k : {16, 64, 256, 4096}) {
        fw_plan p = bestp;
        p.rjs_cap = k;
        float t;
        if ((rc = time_plan(p, &t)) != FW_OK) return rc;
        if (t < bestt) bestt = t, bestp = p;
    }
    // the lanes' shared eRVS threshold: fewer key draws where eRVS scans long rows; taken
    // only when clearly faster (by 2 %), since it changes nothing where eRVS never runs
    {
        fw_plan p = bestp;
        p.rvs_share = 1;
        float t;
        if ((rc = time_plan(p, &t)) != FW_OK) return rc;
        if (t < 0.98f * bestt) bestt = t, bestp = p;
    }
    // eRVS lanes on long rows, for one logic only (hub lanes run in fw_walk launches; a mix
    // is tuned for the batches and servers that take it): P = 128 or 256 on rows of at
    // least 1024 or 8192 entries
    if (n_logics == 1) {
        for (int32_t hl : {128, 256})
            for (int32_t hd : {1024, 8192}) {
                fw_plan p = bestp;
                p.hub_deg = hd;
                p.hub_lanes = hl;
                float t;
                if ((rc = time_plan(p, &t)) != FW_OK) return rc;
                if (t < bestt) bestt = t, bestp = p;
            }
    }
    // the persistent grid: the occupancy limit (0), half of it, and twice it (blocks past
    // the resident ones start as others finish)
    {
        int64_t nw = 0;
        for (int32_t i = 0; i < n_logics; ++i) nw += n;
        const int full = fw::walk_grid(logics[0].kind, logics[0].weighted && g->h, batched, bestp.lds_cap, nw);
        for (int gr : {full / 2, full * 2}) {
            if (gr < 1) continue;
            fw_plan p = bestp;
            p.grid = gr;
            float t;
            if ((rc = time_plan(p, &t)) != FW_OK) return rc;
            if (t < bestt) bestt = t, bestp = p;
        }
    }
    *out = bestp;
    return ok();
}

struct fw_batch {
    fw_graph *g = nullptr;
    fw::WalkArgs a;
    int kind = 0;
    bool weighted = false;
    int grid = 1;
    fw::QueryDev *d_queries = nullptr;
    unsigned long long *d_queue = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static void batch_free(fw_batch *b)
{
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    (void)hipFree(b->d_queries);
    (void)hipFree(b->d_queue);
    delete b;
}

// Checks query i of a batch and fills its device-table entry; `first` is the flattened
// index of its first walker.
static int query_entry(const fw_graph *g, const fw_plan *pl, const fw_query *qs, int64_t i, const int32_t *starts,
                       int64_t starts_len, int32_t *paths, int64_t paths_len, int32_t *lengths, int64_t lengths_len,
                       int64_t first, fw::QueryDev &d)
{
    const fw_query &q = qs[i];
    int rc;
    if ((rc = check_logic(g, &q.logic)) != FW_OK) return rc;
    if ((rc = check_bound(g, pl, &q.logic)) != FW_OK) return rc;
    if (q.logic.kind != qs[0].logic.kind || (q.logic.weighted != 0) != (qs[0].logic.weighted != 0))
        return fail(FW_E_INVALID, "batch: all queries of a batch share kind and weighting");
    if (q.n < 0 || q.n >= ((int64_t)1 << 31)) return fail(FW_E_INVALID, "query %lld: n out of range", (long long)i);
    if (q.L < 0 || q.L >= (1 << 20)) return fail(FW_E_INVALID, "query %lld: L out of range", (long long)i);
    if (q.start_off < 0 || q.out_off < 0 || q.len_off < 0)
        return fail(FW_E_INVALID, "query %lld: negative offset", (long long)i);
    if (q.n > 0 && (!starts || !paths || !lengths)) return fail(FW_E_INVALID, "batch: null starts/paths/lengths");
    // every block the query addresses must lie inside the caller's arrays
    if (q.start_off + q.n > starts_len || q.len_off + q.n > lengths_len ||
        q.out_off + q.n * ((int64_t)q.L + 1) > paths_len)
        return fail(FW_E_INVALID, "query %lld: its starts/paths/lengths block exceeds the given array", (long long)i);
    fill_query(&q.logic, d);
    d.first = first;
    d.n = q.n;
    d.starts = starts ? starts + q.start_off : nullptr;
    d.paths = paths ? paths + q.out_off : nullptr;
    d.lengths = lengths ? lengths + q.len_off : nullptr;
    d.L = q.L;
    d.key0 = (uint32_t)q.seed;
    d.key1 = (uint32_t)(q.seed >> 32);
    return FW_OK;
}

int fw_batch_create(fw_graph *g, const fw_query *qs, int64_t nq, const fw_plan *pl, int32_t strategy,
                    const int32_t *starts, int64_t starts_len, int32_t *paths, int64_t paths_len, int32_t *lengths,
                    int64_t lengths_len, fw_batch **out)
{
    if (!g || !pl || !out || (nq > 0 && !qs)) return fail(FW_E_INVALID, "fw_batch_create: null argument");
    if (nq < 0 || nq >= ((int64_t)1 << 31)) return fail(FW_E_INVALID, "fw_batch_create: nq must be in [0, 2^31)");
    if (!fw::valid_strategy(strategy))
        return fail(FW_E_INVALID, "fw_batch_create: bad strategy %d", strategy);
    int rc = check_plan(pl);
    if (rc != FW_OK) return rc;
    if (pl->hub_deg > 0 && pl->hub_lanes != 64)
        return fail(FW_E_INVALID, "fw_batch_create: hub lanes (hub_lanes > 64) apply to fw_walk launches only");
    std::vector<fw::QueryDev> tab((size_t)(nq > 0 ? nq : 1));
    int64_t total = 0;
    for (int64_t i = 0; i < nq; ++i) {
        if ((rc = query_entry(g, pl, qs, i, starts, starts_len, paths, paths_len, lengths, lengths_len, total,
                              tab[(size_t)i])) != FW_OK)
            return rc;
        total += qs[i].n;
    }
    const bool weighted = nq > 0 && qs[0].logic.weighted && g->h;
    if (weighted && strategy != FW_RVS_ONLY && !g->prepped)
        return fail(FW_E_STATE, "fw_batch_create: call fw_graph_preprocess before a weighted eRJS/AUTO batch");
    HIP_TRY(hipSetDevice(g->device));
    fw_batch *b = new fw_batch();
    b->g = g;
    if (hipMalloc((void **)&b->d_queries, sizeof(fw::QueryDev) * tab.size()) != hipSuccess ||
        hipMalloc((void **)&b->d_queue, sizeof(unsigned long long)) != hipSuccess) {
        batch_free(b);
        return fail(FW_E_NOMEM, "fw_batch_create: hipMalloc failed");
    }
    if (hipMemcpy(b->d_queries, tab.data(), sizeof(fw::QueryDev) * tab.size(), hipMemcpyHostToDevice) != hipSuccess) {
        batch_free(b);
        return fail(FW_E_DEVICE, "fw_batch_create: hipMemcpy failed");
    }
    if (nq > 0) fill_args(g, &qs[0].logic, b->a);
    else memset(&b->a, 0, sizeof(b->a));
    plan_args(pl, strategy, b->a);
    b->a.n = total;
    b->a.queue = b->d_queue;
    b->a.err = (int *)(g->scratch + 1);
    b->a.queries = b->d_queries;
    b->a.nq = (int32_t)nq;
    b->kind = nq > 0 ? qs[0].logic.kind : FW_NODE2VEC;
    b->weighted = weighted;
    b->grid = pl->grid > 0 ? pl->grid : fw::walk_grid(b->kind, weighted, true, pl->lds_cap, total);
    *out = b;
    return ok();
}

int fw_batch_launch(fw_batch *b, uint64_t *stats, void *stream)
{
    if (!b) return fail(FW_E_INVALID, "fw_batch_launch: null batch");
    if (b->a.n == 0) return ok();
    fw::WalkArgs a = b->a;
    a.stats = (unsigned long long *)stats;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(fw::launch_zero(b->d_queue, 1, s));
    HIP_TRY(fw::launch_walk(a, b->kind, b->weighted, true, b->grid, s));
    return ok();
}

int fw_batch_capture(fw_batch *b, uint64_t *stats, void *stream)
{
    if (!b) return fail(FW_E_INVALID, "fw_batch_capture: null batch");
    if (!stream) return fail(FW_E_INVALID, "fw_batch_capture: needs a non-null stream");
    hipStream_t s = (hipStream_t)stream;
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const int rc = fw_batch_launch(b, stats, stream);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &graph);
    if (rc != FW_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(FW_E_DEVICE, "fw_batch_capture: %s", hipGetErrorString(e));
    b->graph = graph;
    HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return ok();
}

int fw_batch_replay(fw_batch *b, void *stream)
{
    if (!b || !b->exec) return fail(FW_E_STATE, "fw_batch_replay: no captured graph");
    HIP_TRY(hipGraphLaunch(b->exec, (hipStream_t)stream));
    return ok();
}

int fw_batch_destroy(fw_batch *b)
{
    batch_free(b);
    return ok();
}

}  // extern "C"

// ---------------------------------------------------------------- allocation-free batch
// Scratch of fw_batch_run_noalloc: the walker counter in the first 256 bytes, then the
// query table.  One copy per device for the life of the process; in host code this name
// is only a stand-in for the symbol, the device address comes from hipGetSymbolAddress.
static_assert(sizeof(fw::QueryDev) == 176, "the scratch size stated in flexiwalk.h assumes 176-byte query entries");
static __device__ __align__(256) unsigned char scratch[256 + FW_NOALLOC_MAX_QUERIES * sizeof(fw::QueryDev)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's scratch, looked up once per device.
int scratch_of(int dev, unsigned char **out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(FW_E_DEVICE, "fw_batch_run_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(FW_E_DEVICE, "fw_batch_run_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = (unsigned char *)p;
    }
    *out = g_scratch_ptr[dev];
    return ok();
}
}  // namespace

extern "C" {

int fw_batch_run_noalloc(fw_graph *g, const fw_query *qs, int64_t nq, const fw_plan *pl, int32_t strategy,
                         const int32_t *starts, int64_t starts_len, int32_t *paths, int64_t paths_len,
                         int32_t *lengths, int64_t lengths_len, uint64_t *stats, void *stream)
{
    if (!g || !pl || (nq > 0 && !qs)) return fail(FW_E_INVALID, "fw_batch_run_noalloc: null argument");
    if (nq < 0 || nq > FW_NOALLOC_MAX_QUERIES)
        return fail(FW_E_INVALID, "fw_batch_run_noalloc: nq = %lld, must be in [0, %d]", (long long)nq,
                    FW_NOALLOC_MAX_QUERIES);
    if (!fw::valid_strategy(strategy)) return fail(FW_E_INVALID, "fw_batch_run_noalloc: bad strategy %d", strategy);
    int rc = check_plan(pl);
    if (rc != FW_OK) return rc;
    if (pl->hub_deg > 0 && pl->hub_lanes != 64)
        return fail(FW_E_INVALID, "fw_batch_run_noalloc: hub lanes (hub_lanes > 64) apply to fw_walk launches only");
    // every query is checked before anything is written to the device
    int64_t total = 0;
    for (int64_t i = 0; i < nq; ++i) {
        fw::QueryDev d;
        if ((rc = query_entry(g, pl, qs, i, starts, starts_len, paths, paths_len, lengths, lengths_len, total, d)) !=
            FW_OK)
            return rc;
        total += qs[i].n;
    }
    const bool weighted = nq > 0 && qs[0].logic.weighted && g->h;
    if (weighted && strategy != FW_RVS_ONLY && !g->prepped)
        return fail(FW_E_STATE, "fw_batch_run_noalloc: call fw_graph_preprocess before a weighted eRJS/AUTO batch");
    if (total == 0) return ok();
    HIP_TRY(hipSetDevice(g->device));
    unsigned char *sp = nullptr;
    if ((rc = scratch_of(g->device, &sp)) != FW_OK) return rc;
    auto *queue = (unsigned long long *)sp;
    auto *tab = (fw::QueryDev *)(sp + 256);
    hipStream_t s = (hipStream_t)stream;
    // the table goes up in chunks staged on this thread's stack (pageable memory: each
    // copy has read its source when it returns)
    constexpr int kChunk = 32;
    fw::QueryDev chunk[kChunk];
    int64_t first = 0;
    for (int64_t i0 = 0; i0 < nq; i0 += kChunk) {
        const int m = (int)std::min<int64_t>(kChunk, nq - i0);
        for (int k = 0; k < m; ++k) {
            (void)query_entry(g, pl, qs, i0 + k, starts, starts_len, paths, paths_len, lengths, lengths_len, first,
                              chunk[k]);
            first += qs[i0 + k].n;
        }
        HIP_TRY(hipMemcpyAsync(tab + i0, chunk, sizeof(fw::QueryDev) * (size_t)m, hipMemcpyHostToDevice, s));
    }
    fw::WalkArgs a;
    fill_args(g, &qs[0].logic, a);
    plan_args(pl, strategy, a);
    a.n = total;
    a.stats = (unsigned long long *)stats;
    a.queue = queue;
    a.err = (int *)(g->scratch + 1);
    a.queries = tab;
    a.nq = (int32_t)nq;
    const int grid = pl->grid > 0 ? pl->grid : fw::walk_grid(qs[0].logic.kind, weighted, true, pl->lds_cap, total);
    HIP_TRY(fw::launch_zero(queue, 1, s));
    HIP_TRY(fw::launch_walk(a, qs[0].logic.kind, weighted, true, grid, s));
    return ok();
}

}  // extern "C"
