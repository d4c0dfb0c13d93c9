// Internal declarations shared by the kernels (fw_kernels.hip) and the C ABI layer
// (fw_api.hip).  Not installed; the public interface is include/flexiwalk.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fw {

enum Kind : int { kNode2Vec = 1, kMetaPath = 2 };
enum Strategy : int { kAuto = 0, kRvsOnly = 1, kRjsOnly = 2 };
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
constexpr int kDefaultLdsCap = 2048; // int32 entries of N(prev) per wavefront
constexpr int kRjsPerRound = 4;      // eRJS trials a lane runs between eRVS services

// Everything a walk launch reads.  Float constants are prepared on the host in float32
// so that the device and every other float32 evaluation agree bit for bit.
struct WalkArgs {
    const int64_t *row_ptr;
    const int32_t *col;
    const float *h;
    const uint8_t *label;
    const float *hmax;
    const float *hsum;
    int64_t nv;

    const int32_t *starts;
    int64_t n;
    int32_t L;
    int32_t *paths;
    int32_t *lengths;
    unsigned long long *stats;  // may be null
    unsigned long long *queue;  // next walker to hand out
    int *err;                   // set to 1 on an out-of-range start

    uint32_t key0, key1;        // Philox key = seed
    float inv_p, inv_q;         // 1/p, 1/q
    float lo_w, hi_w;           // min(1, 1/q), max(1, 1/q)
    float wmax0, wavg0;         // max and mean workload weight at step 0
    float wmax1, wavg1;         // ... at steps >= 1
    float rho;
    int32_t d_lo;
    int32_t rjs_cap;
    int32_t strategy;
    int32_t lds_cap;
    int32_t schema_len;
    uint8_t schema[64];
    int32_t item_bytes;         // col (+ h) (+ label) per scanned or proposed edge
};

hipError_t launch_walk(const WalkArgs &a, int kind, bool weighted, int grid, hipStream_t s);
hipError_t launch_zero(unsigned long long *p, int n, hipStream_t s);
hipError_t launch_preprocess(const int64_t *row_ptr, const float *h, int64_t nv, float *hmax, float *hsum,
                             hipStream_t s);
hipError_t launch_validate_rows(const int64_t *row_ptr, int64_t nv, int64_t ne, int *err, hipStream_t s);
hipError_t launch_validate_edges(const int64_t *row_ptr, const int32_t *col, const float *h, int64_t nv,
                                 int *err, unsigned long long *max_deg, hipStream_t s);
hipError_t launch_profile(const WalkArgs &a, int kind, bool weighted, bool rjs_style, const int32_t *nodes,
                          int nsample, int per_node, float *sink, hipStream_t s);
int walk_grid(int kind, bool weighted, int lds_cap, int64_t n);

}  // namespace fw
