// Internal declarations shared by the kernels (fw_kernels.hip) and the C ABI layer
// (fw_api.hip).  Not installed; the public interface is include/flexiwalk.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fw {

enum Kind : int { kNode2Vec = 1, kMetaPath = 2, kSecondPR = 3 };
constexpr int kNumKinds = 3;

// Logics whose weight depends on u in N(prev) (the membership test).
__host__ __device__ constexpr bool uses_membership(int kind) { return kind == kNode2Vec || kind == kSecondPR; }
enum Strategy : int { kAuto = 0, kRvsOnly = 1, kRjsOnly = 2, kRandomSelect = 4, kDegreeSelect = 5 };

__host__ __device__ constexpr bool valid_strategy(int s)
{
    return s == kAuto || s == kRvsOnly || s == kRjsOnly || s == kRandomSelect || s == kDegreeSelect;
}
enum Stat : int {
    kStSteps = 0,
    kStRjs = 1,
    kStRvs = 2,
    kStFallback = 3,
    kStTrials = 4,
    kStTriggers = 5,
    kStEarly = 6,
    kStBytes = 7,
    kNumStats = 8
};

constexpr int kBlock = 256;          // 4 wavefronts per block, each independent
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kDefaultLdsCap = 512;  // int32 entries of N(prev) per wavefront: with the four 1 KB vertex-record
                                     // slots a block takes 24 KB, six blocks per CU (1024: 32 KB blocks, slower)
// eRJS proposals whose loads a lane issues together.  Only depth 3 is built: a build with
// depth 4 whose counted launches were compiled for 5 waves per SIMD (heavy spills) left the
// oracle's path after eRJS cap fall-backs, and that failure has no identified cause, so no
// other depth may be built until one is found.
#ifndef FW_RJS_BATCH
#define FW_RJS_BATCH 3
#endif
#if FW_RJS_BATCH != 3
#error "FW_RJS_BATCH: only the eRJS load batch of depth 3 has passed the parity suite"
#endif
constexpr int kRjsBatch = FW_RJS_BATCH;
// h-proportional proposal record per CSR entry, 64 bytes (one DRAM line holds it whole):
//   {col_k, bits(h_k), col_a, bits(h_a)}, {threshold, label_k | label_a << 8, 0, 0},
//   vrec[col_k], vrec[col_a]  (the candidates' vertex records for the next step's set-up)
constexpr int kPropU4 = 4;
#ifndef FW_MERGE_RATIO
#define FW_MERGE_RATIO 8
#endif
constexpr int kMergeRatio = FW_MERGE_RATIO;  // eRVS merges N(v) with N(prev) while d(prev) <= this * d(v)
#ifndef FW_MIN_WAVES
#define FW_MIN_WAVES 5
#endif
#ifndef FW_MIN_WAVES_BATCH
#define FW_MIN_WAVES_BATCH 4
#endif
// resident waves per SIMD the walk kernel is compiled for: single-query launches at 5 (96
// VGPRs; the extra wave hides more memory latency than the few spills cost), batched and
// resumable ones at 4 (their per-query state spills more at 96).  Launches that keep the
// device counters are compiled for 4 waves, fixed: their extra state spills heavily at 96,
// and the one build that did so is the unexplained parity failure noted at kRjsBatch (the
// persistent grid is sized by the counter-free variant; blocks beyond what is resident
// start late and find the walker queue drained)
constexpr int kMinWaves = FW_MIN_WAVES;
constexpr int kMinWavesBatch = FW_MIN_WAVES_BATCH;
constexpr int kMinWavesCounted = 4;
// the eRVS-only variant (no eRJS code) fits 6 waves in its registers without spills
constexpr int kMinWavesRvsOnly = 7;

// Per-query constants of a walk job.  Float constants are prepared on the host in float32
// exactly as the definition states, so every float32 evaluation agrees bit for bit.
// A single-query launch carries one of these in its kernel arguments; a batched launch
// reads them from a device table indexed by query.
struct QueryDev {
    int64_t first;              // first flattened walker index of the query
    int64_t n;                  // walkers
    const int32_t *starts;      // n start vertices
    int32_t *paths;             // n * (L + 1) path slots
    int32_t *lengths;           // n lengths
    uint32_t key0, key1;        // Philox key = the query's seed
    float inv_p, inv_q;         // 1/p, 1/q
    float lo_w, hi_w;           // min(1, 1/q), max(1, 1/q)
    float wmax0, wavg0;         // max and mean workload weight at step 0
    float wmax1, wavg1;         // ... at steps >= 1 (Node2Vec, MetaPath)
    float gamma, omg;           // second-order PageRank: gamma and 1 - gamma
    int32_t L;
    int32_t schema_len;
    uint8_t schema[64];
    // resumable walks (served form): prog[i] = steps done so far, or kDone when the walk
    // has finished; done counts finished walkers.  Null for one-shot launches.
    int32_t *prog;
    int32_t *done;
};

constexpr int32_t kDone = INT32_MIN;

// Device layout of a graph.  Besides the caller's CSR the library keeps
//   edges[k] = {col[k], bits(h[k])}: one 8-byte load per proposed or scanned edge;
//   erec8[k] = col[k] | code[k] << 24 instead, for 8-bit weights on graphs of at most
//              2^24 vertices: one 4-byte load, h = h_scale * code;
//   vrec[v]  = {low 32 bits of row start, degree, bits(h_MAX[v]), bits(h_SUM[v])}:
//              one 16-byte load per step set-up;
//   start_hi[v] = high 32 bits of the row start (only when ne >= 2^32, else null);
//   col (alone) for the membership search and LDS staging of N(prev).
struct WalkArgs {
    const uint2 *edges;         // null when erec8 holds the edges
    const uint32_t *erec8;      // 8-bit weights: {col | code << 24} per entry, or null
    float h_scale;              // 8-bit weights: h = h_scale * code
    const uint4 *vrec;
    const uint32_t *start_hi;
    const int32_t *col;
    const uint8_t *label;
    int64_t nv;

    int64_t n;                  // walkers in the launch (all queries)
    unsigned long long *stats;  // may be null
    unsigned long long *queue;  // next walker to hand out
    int *err;                   // set to 1 on an out-of-range start
    float rho;
    int32_t d_lo;
    int32_t rjs_cap;
    int32_t strategy;
    int32_t lds_cap;
    int32_t item_bytes;         // col (+ h) (+ label) per scanned or proposed edge
    int32_t tick_steps;         // resumable walks: steps per walker per launch
    int32_t bound;              // 1: Node2Vec split eRJS bound (symmetric graphs only)
    const uint4 *mtab;          // edge index (8 uint4 per bucket) or null: search the sorted rows
    const uint4 *prop;          // proposal records (kPropU4 uint4 per entry) or null
    int32_t proposal;           // 1: h-proportional eRJS proposals through `prop`; 2: as 1, and
                                // MetaPath proposes within the wanted label's group (`lprop`)
    const int64_t *lrow;        // label groups: first grouped position of (v, l) at v * nlab + l
    const uint4 *lprop;         // proposal records of the label groups (kPropU4 uint4 per entry)
    int32_t nlab;               // labels 0 .. nlab - 1 have groups
    int32_t hub_deg;            // eRVS rows of at least this degree use hub_v * 64 lanes (0: never)
    int32_t hub_v;              // virtual lanes per lane there: 1, 2 or 4
    int32_t rvs_share;          // 1: eRVS lanes take the largest threshold after a round with a jump event
    uint64_t mtab_mask;         // buckets - 1

    QueryDev q0;                // the query of a single-query launch
    const QueryDev *queries;    // batched launch: nq entries, ascending `first`
    int32_t nq;
};

hipError_t launch_walk(const WalkArgs &a, int kind, bool weighted, bool batch, int grid, hipStream_t s);
hipError_t launch_zero(unsigned long long *p, int n, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
// 8-bit weights: h[k] = h_scale * code[k] (float32 product) for k < ne.
hipError_t launch_dequantize(const uint8_t *code, float h_scale, int64_t ne, float *h, hipStream_t s);
// 8-bit weights: erec8[k] = col[k] | code[k] << 24 for k < ne (every col < 2^24).
hipError_t launch_pack8(const int32_t *col, const uint8_t *code, int64_t ne, uint32_t *erec8, hipStream_t s);
hipError_t launch_layout(const int64_t *row_ptr, const int32_t *col, const float *h, int64_t nv, int64_t ne,
                         uint2 *edges, uint4 *vrec, uint32_t *start_hi, hipStream_t s);
hipError_t launch_preprocess(const int64_t *row_ptr, const float *h, int64_t nv, uint4 *vrec, hipStream_t s);
// Proposal records of h-proportional eRJS: Walker's alias table per row (the sweeping
// construction in exact integer arithmetic, in parallel form: a scan pass and a merge
// pass, one wave per row) written as prop[4k] = {col[k], h[k], col[a], h[a]},
// prop[4k+1] = {threshold, lab[k] | lab[a] << 8, a, 0}, prop[4k+2..3] = vrec of col[k],
// col[a].  Scratch: val (16 bytes) and idx (4 bytes) per entry, rowinfo (16 bytes) per row.
// rmax: each row's h maximum, or null to take it from vrec[row] (rows are vertices).
// Rows longer than 8192 entries are merged one thread per entry (hubs: nv int32 of
// scratch, nhub: one int).
hipError_t launch_build_alias(const int64_t *row_ptr, const int32_t *col, const float *h, const uint8_t *label,
                              int64_t nv, const uint4 *vrec, const float *rmax, uint4 *val, int32_t *idx,
                              ulonglong2 *rowinfo, int32_t *hubs, int *nhub, uint4 *prop, hipStream_t s);
// Labels of a graph with label groups: at most this many (0 .. kMaxLabels - 1).
constexpr int kMaxLabels = 16;
// *out = the largest of label[0 .. ne) (atomicMax into *out, which starts at 0).
hipError_t launch_label_max(const uint8_t *label, int64_t ne, int *out, hipStream_t s);
// Label groups of every row (nlab <= kMaxLabels labels, each below nlab): lrow[v * nlab + l]
// = row_ptr[v] + the entries of row v with a smaller label, gmax[v * nlab + l] = the largest
// h of group (v, l) (0 when empty; 1 when h is null), and the entries in grouped order:
// vcol, vh (when h is non-null) and vlab at position lrow[v * nlab + l] + (rank among the
// row's label-l entries).  lrow[nv * nlab] is not written.
hipError_t launch_label_groups(const int64_t *row_ptr, const int32_t *col, const float *h, const uint8_t *label,
                               int64_t nv, int nlab, int64_t *lrow, float *gmax, int32_t *vcol, float *vh,
                               uint8_t *vlab, hipStream_t s);
// thr[k] = threshold and alias[k] = alias offset of proposal record k, for k < ne.
hipError_t launch_export_alias(const uint4 *prop, int64_t ne, uint32_t *thr, int32_t *alias, hipStream_t s);
// Edge index: inserts every entry (v, col[k]) of the rows with its h (1 when h is null) into
// `tab` (buckets of 8 keys and 8 h, 128 bytes each, keys all kEmptyKey on entry;
// buckets = mask + 1, a power of two, at least a quarter of ne).
hipError_t launch_build_index(const int64_t *row_ptr, const int32_t *col, const float *h, int64_t nv,
                              unsigned long long *tab, uint64_t mask, hipStream_t s);
// blocks * kBlock lanes each read 4 * rounds random 8-byte records of a[0, mask] (mask + 1 a
// power of two).
hipError_t launch_random_reads(const uint2 *a, uint64_t mask, int blocks, int rounds, unsigned *sink, hipStream_t s);
// Sets bit 4 of *err unless every entry (v, u) has a reverse (u, v) with the same h.
// Rows must already be validated (in range, strictly ascending).
hipError_t launch_check_symmetry(const int64_t *row_ptr, const int32_t *col, const float *h, int64_t nv, int *err,
                                 hipStream_t s);
hipError_t launch_validate_rows(const int64_t *row_ptr, int64_t nv, int64_t ne, int *err, hipStream_t s);
hipError_t launch_validate_edges(const int64_t *row_ptr, const int32_t *col, const float *h, int64_t nv,
                                 int *err, unsigned long long *max_deg, hipStream_t s);
hipError_t launch_profile(const WalkArgs &a, int kind, bool weighted, bool rjs_style, const int32_t *nodes,
                          int nsample, int per_node, float *sink, hipStream_t s);
// {vertex k * stride, its degree} for k < n (stride * (n - 1) < nv).
hipError_t launch_profile_pick(const int64_t *row_ptr, int64_t stride, int n, int2 *out, hipStream_t s);
// Persistent grid filling the device: resident blocks per CU (of the counter-free kernel
// variant the launch takes: batched, eRVS-only (strategy FW_RVS_ONLY, single query) or the
// general one) times the CUs, at most one block per 256 walkers.
int walk_grid(int kind, bool weighted, bool batch, int lds_cap, int64_t n, bool rvs_only = false);

}  // namespace fw
