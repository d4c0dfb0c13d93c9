// Host-side internals shared by the C ABI (fw_api.hip) and the walk server
// (fw_server.hip): the graph object, error reporting and launch-argument helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/flexiwalk.h"
#include "fw_internal.h"

// Library-owned device copy of a graph (opaque to callers).
struct fw_graph {
    int device = 0;
    int64_t nv = 0, ne = 0, max_deg = 0;
    int64_t *row_ptr = nullptr;
    int32_t *col = nullptr;
    float *h = nullptr;
    uint8_t *label = nullptr;
    uint2 *edges = nullptr;                 // {col, bits(h)} per entry, or null when erec8 holds the edges
    uint32_t *erec8 = nullptr;              // 8-bit weights: {col | code << 24} per entry (nv <= 2^24), or null
    float h_scale = 0.0f;                   // 8-bit weights: h = h_scale * code
    bool q8 = false;                        // the weights came as 8-bit codes
    uint4 *vrec = nullptr;                  // {start_lo, degree, bits(h_MAX), bits(h_SUM)} per vertex
    uint32_t *start_hi = nullptr;           // high row-start bits, only when ne >= 2^32
    unsigned long long *scratch = nullptr;  // [0] walker queue, [1] error flag (int)
    bool prepped = false;
    bool symmetric = false;                 // every (v, u) has a reverse (u, v) with equal h
    unsigned long long *mtab = nullptr;     // edge index: 128-byte buckets of 8 keys v << 32 | u and their h, or null
    uint4 *prop = nullptr;                  // h-proportional proposal records (kPropU4 uint4 per entry), or null
    int64_t *lrow = nullptr;                // label groups: first grouped position of (v, l) at v * nlab + l, or null
    uint4 *lprop = nullptr;                 // proposal records of the label groups (grouped order), or null
    int32_t nlab = 0;                       // label groups exist for labels 0 .. nlab - 1
    uint64_t mtab_mask = 0;                 // buckets - 1
};

namespace fw {
constexpr int kMaxLdsCap = 8192;  // four waves' N(prev) staging stays within a CU's 160 KB of LDS

namespace host {

// Record a message for fw_last_error (this thread) and return `code`.
int fail(int code, const char *fmt, ...);
// Clear the message and return FW_OK.
int ok();

int check_logic(const fw_graph *g, const fw_logic *lg);
int check_plan(const fw_plan *pl);
// plan.bound = 1 or 2 for Node2Vec needs a symmetric graph
int check_bound(const fw_graph *g, const fw_plan *pl, const fw_logic *lg);
// Per-query float constants of a logic, in float32 exactly as the definition states.
void fill_query(const fw_logic *lg, QueryDev &q);
// Graph fields and logic-derived fields of a launch.
void fill_args(const fw_graph *g, const fw_logic *lg, WalkArgs &a);
void plan_args(const fw_plan *pl, int32_t strategy, WalkArgs &a);

}  // namespace host
}  // namespace fw

#define HIP_TRY(expr)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return fw::host::fail(FW_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));             \
    } while (0)
