// gfx950 kernels of the dynamic random-walk sampler.
//
// walk_kernel is the runtime kernel of FlexiWalker (arXiv 2512.00705, Section 5,
// "Concurrent Rejection and Reservoir Sampling" and "Dynamic Query Scheduling")
// re-designed for wave64:
//   * every lane owns one walker and runs the cost model of Section 4.1 (Eq. runtime)
//     at each step; eRJS (Section 3.3) runs inside the lane;
//   * a 64-bit ballot collects the lanes whose step needs eRVS (Section 3.2); the whole
//     wave serves them one at a time, the lane's state broadcast with readlane;
//   * eRVS keys the first 64 neighbours (Algorithm 1 in the log domain), takes a wave
//     maximum, then each lane scans its strided neighbours with the jump of Eq. (jump)
//     and a final wave argmax picks the next vertex;
//   * walkers are handed out from a global counter, one atomic per wave refill.
// The membership test u in N(prev) (Node2Vec, second-order PageRank) is, in eRJS, one
// bucket of the edge index (or an interpolation search of prev's sorted row) and only
// when the bounds of w~ leave the test open; in eRVS, where the whole wave tests one row,
// a bisection of N(prev) staged in LDS when short enough.  Random reads are what this
// kernel pays for (each costs a DRAM line), so an edge is one 8-byte record {col, h}
// (4 bytes with 8-bit weights), a vertex one 16-byte record {start, degree, h_MAX, h_SUM},
// and an h-proportional proposal one 64-byte record that also holds the vertex records
// of its two candidates.  Optional eRJS boards (split bound, member board; extensions of
// Section 3.3) cut the expected trials; see walk_kernel.
#include "fw_device.h"
#include "fw_internal.h"

namespace fw {

enum Mode : int { kIdle = 0, kSetup = 1, kRjs = 2, kRvs = 3, kAdv = 4 };

// Dynamic LDS of a walk block: each wave's four slots of 64 vertex records filled by LDS DMA
// from proposal records, then each wave's N(prev) staging area (lds_cap int32).
// Dynamic LDS of a walk block: per wave, four slots of 64 vertex records (eRJS proposals'
// candidates; not in the eRVS-only variant, rvs_only) and lds_cap entries of N(prev).
static size_t walk_lds_bytes(int lds_cap, bool rvs_only = false)
{
    return (size_t)kWavesPerBlock * (size_t)lds_cap * sizeof(int32_t) +
           (rvs_only ? 0 : (size_t)kWavesPerBlock * 4 * kWave * 16);
}

// An LDS address for the LDS-DMA load builtin (the pointer must lie in this block's LDS).
__device__ __forceinline__ __attribute__((address_space(3))) void *lds_ptr(uint4 *p)
{
    return (__attribute__((address_space(3))) void *)p;
}

// N(prev) for the membership test: a copy in this wave's LDS or the row of prev in col,
// read through one flat pointer either way.  `indexed`: lanes test different rows (eRJS
// style); an unstaged row then goes through the edge index when the graph has one, else
// an interpolation search (fewest probes per lane).  Otherwise the whole wave tests one
// row (an eRVS step): its probes hit the cache, and a branch-free bisection, whose trip
// count is the same in every lane, beats a search that is cheaper on average but waits
// for its slowest lane.
struct Mem {
    const int32_t *p;
    int64_t len;
    bool staged;
    bool indexed;
};

// u in N(prev): LDS copy, else the edge index if asked for, else a search of the row.
__device__ __forceinline__ bool in_prev_row(const WalkArgs &a, const Mem &m, int32_t prev, int32_t u)
{
    if (m.indexed) {
        if (!m.staged && a.mtab != nullptr) return index_contains(a.mtab, a.mtab_mask, prev, u);
        return sorted_contains_interp(m.p, (int32_t)m.len, u, (int32_t)a.nv);
    }
    return sorted_contains_bisect(m.p, (int32_t)m.len, u);
}

// The constants of query q: a device table for batched launches, the kernel argument
// block otherwise.
template <bool BATCH>
__device__ __forceinline__ const QueryDev &query(const WalkArgs &a, int32_t q)
{
    return BATCH ? a.queries[q] : a.q0;
}

// Query holding flattened walker w: the last one whose first walker is <= w.
__device__ __forceinline__ int32_t query_of(const WalkArgs &a, int64_t w)
{
    int32_t lo = 0, hi = a.nq - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (a.queries[mid].first <= w) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The workload weights of a step that depend on u only through u in N(prev): `mem` for
// u in N(prev), `oth` otherwise, `ret` for u = prev, and their smallest and largest
// (Node2Vec: 1, 1/q, 1/p from the query; second-order PageRank: the two branches of
// Eq. (2ndpr) at this step's d(v), d(v'), the return taking the second).
struct StepW {
    float mem, oth, ret, lo, hi;
};

template <int KIND>
__device__ __forceinline__ StepW step_weights(const QueryDev &Q, int32_t dv, int32_t dvp)
{
    if (KIND == kSecondPR) {
        // in float32 in the order of Eq. (2ndpr): ((1-g)/d(v) + g/d(v')) * max_d, ((1-g)/d(v)) * max_d
        const float t1 = Q.omg / (float)dv;
        const float t2 = Q.gamma / (float)(dvp > 0 ? dvp : 1);
        const float md = (float)(dv > dvp ? dv : dvp);
        const float in = (t1 + t2) * md, out = t1 * md;
        return StepW{in, out, out, fminf(in, out), fmaxf(in, out)};
    }
    return StepW{1.0f, Q.inv_q, Q.inv_p, Q.lo_w, Q.hi_w};
}

// Transition weight w~ = w * h of the edge at CSR position k (record e) at step j
// (Section 2.1, Eq. prob; Eq. node2vec; MetaPath rule; Eq. 2ndpr).  `m` holds N(prev)
// sorted; `sw` the step's weights.
template <int KIND, bool W>
__device__ __forceinline__ float edge_weight(const WalkArgs &a, const QueryDev &Q, int64_t k, uint2 e, int j,
                                             int32_t prev, const Mem &m, uint8_t want, const StepW &sw)
{
    const float hv = W ? __uint_as_float(e.y) : 1.0f;
    if (KIND == kSecondPR) {
        if (j == 0) return hv;
        const int32_t u = (int32_t)e.x;
        if (u == prev) return sw.ret * hv;
        return in_prev_row(a, m, prev, u) ? sw.mem * hv : sw.oth * hv;
    }
    if (KIND == kNode2Vec) {
        if (j == 0) return hv;
        const int32_t u = (int32_t)e.x;
        if (u == prev) return Q.inv_p * hv;
        return in_prev_row(a, m, prev, u) ? hv : Q.inv_q * hv;
    } else {
        return a.label[k] == want ? hv : 0.0f;
    }
}

// The {col, bits(h)} record of CSR entry k: the 8-byte record, or the 4-byte record of an
// 8-bit-weight graph decoded (h = h_scale * code, one float32 product).
__device__ __forceinline__ uint2 edge_rec(const WalkArgs &a, int64_t k)
{
    if (a.erec8 != nullptr) {
        const uint32_t x = a.erec8[k];
        return make_uint2(x & 0xFFFFFFu, __float_as_uint((float)(x >> 24) * a.h_scale));
    }
    return a.edges[k];
}

// Store the n held path slots p0.. at dst (walk ended or suspended).
__device__ __forceinline__ void flush_path(int32_t *dst, int32_t n, int32_t p0, int32_t p1, int32_t p2)
{
    dst[0] = p0;
    if (n > 1) dst[1] = p1;
    if (n > 2) dst[2] = p2;
}

__device__ __forceinline__ int64_t row_start(const WalkArgs &a, uint4 r, int32_t v)
{
    return a.start_hi ? (int64_t)(((uint64_t)a.start_hi[v] << 32) | r.x) : (int64_t)r.x;
}

// u in N(prev) for the 64 items of one eRVS round, all lanes together: the round's items
// are consecutive entries of cur's sorted row, so the wave merges them with N(prev)
// (sorted, m.p[0, m.len)): it loads the next 64 entries of N(prev) from the wave's cursor
// `lo` (one coalesced load), each lane finds its item among them by a bisection over the
// lanes (ds_bpermute), and the block advances while some item lies beyond it.  The cursor
// then moves past everything below the round's largest item.  Over a whole scan this
// reads N(prev) once, in order, where a search per item costs log d(prev) dependent loads.
// A round whose largest item lies below the entry at the cursor holds no member and
// leaves the cursor where it is: it needs no bisection (the usual round of a hub row
// scanned from a short N(prev)).
// `valid`: the lane holds an item; every lane must call this.
__device__ __forceinline__ bool merge_member(const Mem &m, int32_t u, bool valid, int64_t &lo)
{
    const int lane = lane_id();
    const uint64_t vm = __ballot(valid);
    if (vm == 0) return false;
    // items are consecutive entries of a sorted row: the largest sits in the last valid lane
    const int32_t umax = __builtin_amdgcn_readlane(u, 63 - __builtin_clzll((unsigned long long)vm));
    bool found = false, done = !valid;
    int32_t c = 0;
    for (bool first = true;; first = false) {
        const int64_t vi = lo + lane;
        const int32_t v = vi < m.len ? m.p[vi] : INT32_MAX;
        if (first && umax < __builtin_amdgcn_readfirstlane(v)) return false;
        c = 0;
#pragma unroll
        for (int s = kWave / 2; s > 0; s >>= 1) {
            const int32_t pv = __shfl(v, c + s - 1, kWave);
            if (pv < u) c += s;
        }
        const int32_t vc = __shfl(v, c & (kWave - 1), kWave);
        const int32_t vlast = __shfl(v, kWave - 1, kWave);
        if (!done) {
            found = c < kWave && vc == u;
            done = u <= vlast;
        }
        if (__ballot(!done) == 0) break;
        lo += kWave;  // every open item lies beyond this whole block
    }
    lo += __shfl(c, kWave - 1, kWave);  // entries below the round's largest item
    return found;
}

// merge_member for the eRVS-only kernel variant, same results.  The block of N(prev) at
// the cursor is loaded before the items are first used (it does not depend on them), so
// that its load overlaps the load of the round's edges instead of following it.  Of the
// block, only entries within [smallest item, largest item] can equal an item; when there
// are few (a hub row scanned against a shorter N(prev): a handful per round), each is
// broadcast from its lane and compared with every item at once, with no LDS round trip;
// otherwise each lane bisects the block as merge_member does.  The cursor then moves past
// every entry up to the largest item (later rounds hold only larger items).  In the other
// kernel variants the register budget is held by the eRJS path, where the longer-lived
// block spilled.
constexpr int kMergeBcast = 8;  // most in-range entries compared by broadcast (8: 2.98 s, 16: 3.01 s, 32: 3.20 s on eRVS-only scale 22)
__device__ __forceinline__ bool merge_member_early(const Mem &m, int32_t u, bool valid, int64_t &lo)
{
    const int lane = lane_id();
    int32_t v = lo + lane < m.len ? m.p[lo + lane] : INT32_MAX;
    const uint64_t vm = __ballot(valid);
    if (vm == 0) return false;
    // items are consecutive entries of a sorted row held by a prefix of the lanes
    const int32_t umin = __builtin_amdgcn_readlane(u, __builtin_ctzll((unsigned long long)vm));
    const int32_t umax = __builtin_amdgcn_readlane(u, 63 - __builtin_clzll((unsigned long long)vm));
    if (umax < __builtin_amdgcn_readfirstlane(v)) return false;
    bool found = false;
    for (;;) {
        const uint64_t inr = __ballot(v >= umin && v <= umax);
        if (__popcll(inr) <= kMergeBcast) {
            for (uint64_t mm = inr; mm != 0; mm &= mm - 1) {
                const int32_t e = __builtin_amdgcn_readlane(v, __builtin_ctzll((unsigned long long)mm));
                found = found || u == e;
            }
        } else {
            int32_t c = 0;
#pragma unroll
            for (int s = kWave / 2; s > 0; s >>= 1) {
                const int32_t pv = __shfl(v, c + s - 1, kWave);
                if (pv < u) c += s;
            }
            const int32_t vc = __shfl(v, c & (kWave - 1), kWave);
            found = found || (c < kWave && vc == u);
        }
        const uint64_t le = __ballot(v <= umax);  // a prefix of the block: entries up to the largest item
        if (~le != 0ull) {
            lo += __popcll(le);
            break;
        }
        lo += kWave;
        v = lo + lane < m.len ? m.p[lo + lane] : INT32_MAX;
    }
    return found && valid;
}

template <bool EARLY>
__device__ __forceinline__ bool merge_member_t(const Mem &m, int32_t u, bool valid, int64_t &lo)
{
    return EARLY ? merge_member_early(m, u, valid, lo) : merge_member(m, u, valid, lo);
}

// Transition weight from the membership of u in N(prev) (the same expression as
// edge_weight, for Node2Vec and second-order PageRank).
template <int KIND, bool W>
__device__ __forceinline__ float weight_of_member(uint2 e, int j, int32_t prev, bool member, const StepW &sw)
{
    const float hv = W ? __uint_as_float(e.y) : 1.0f;
    if (j == 0) return hv;
    if ((int32_t)e.x == prev) return sw.ret * hv;
    return member ? sw.mem * hv : sw.oth * hv;
}

// Shared eRVS threshold (plan rvs_share): after a scan round in which some lane drew a
// key, a lane whose threshold lies below the largest one, g, takes g.  Its remaining skip
// T - S is exponential with rate -thr (no item since its last draw has passed it), so
// scaled by thr / g it is the skip towards the first item whose key beats g; keys below g
// cannot win the argmax.  A lane with no threshold yet (-inf) keeps T = 0.
__device__ __forceinline__ void take_shared_threshold(float &thr, float &T, float &S, float g)
{
    if (thr > -INFINITY && thr < g) {
        T = g >= 0.0f ? INFINITY : ((T - S) * thr) / g;
        S = 0.0f;
        thr = g;
    }
}

// eRVS for one step, all 64 lanes cooperating.  Returns the next vertex or -1 when no
// neighbour has positive weight, with the h of the chosen edge in `hsel`.  `trig`
// receives the number of jump events.  `merge`: find u in N(prev) by merging the rows
// (merge_member) instead of searching `mem` per item.
template <int KIND, bool W, bool EARLY>
__device__ __forceinline__ int32_t rvs_step(const WalkArgs &a, const QueryDev &Q, const Mem &mem, uint32_t wid,
                                            int j, int32_t prev, int64_t base, int64_t deg, uint8_t want,
                                            const StepW &sw, uint32_t &trig, float &hsel, bool merge)
{
    const int lane = lane_id();
    const uint32_t k0 = Q.key0, k1 = Q.key1;
    float key = -INFINITY;
    int32_t bi = -1;
    float ru = 0.5f;
    int64_t mlo = 0;  // merge cursor in N(prev)
    // round 0: lane l keys neighbour l, k = u^(1/w~) kept as log(u) / w~
    const uint2 e0 = lane < deg ? edge_rec(a, base + lane) : make_uint2(0u, 0u);
    const bool mem0 = merge && merge_member_t<EARLY>(mem, (int32_t)e0.x, lane < deg, mlo);
    if (lane < deg) {
        const int64_t k = base + lane;
        const float wt = merge ? weight_of_member<KIND, W>(e0, j, prev, mem0, sw)
                               : edge_weight<KIND, W>(a, Q, k, e0, j, prev, mem, want, sw);
        const U4 x = philox(wid, (uint32_t)j, (uint32_t)lane, 1u, k0, k1);
        key = wt > 0.0f ? ln_f(unit_uniform(x.x0)) / wt : -INFINITY;
        ru = unit_uniform(x.x1);
        bi = lane;
    }
    const float lkg = wave_max(key);
    float thr = lkg;
    float T = (thr == -INFINITY) ? 0.0f : (thr >= 0.0f ? INFINITY : ln_f(ru) / thr);
    float S = 0.0f;
    uint32_t nt = 0;
    // scan: lane l owns neighbours l + 64, l + 128, ...; a key is drawn only where the
    // running weight passes the skip threshold T = log(r) / log(k_thr)
    for (int64_t i0 = kWave; i0 < deg; i0 += kWave) {
        const int64_t i = i0 + lane;
        const uint2 ei = i < deg ? edge_rec(a, base + i) : make_uint2(0u, 0u);
        const bool memi = merge && merge_member_t<EARLY>(mem, (int32_t)ei.x, i < deg, mlo);
        bool drew = false;
        if (i < deg) {
            const int64_t k = base + i;
            const float wt = merge ? weight_of_member<KIND, W>(ei, j, prev, memi, sw)
                                   : edge_weight<KIND, W>(a, Q, k, ei, j, prev, mem, want, sw);
            S = S + wt;
            if (S > T) {
                // key conditioned to beat thr: log u' = log1p(expm1(w~ * thr) * V)
                const U4 x = philox(wid, (uint32_t)j, (uint32_t)i, 1u, k0, k1);
                const float av = wt * thr;
                const float m1 = expm1_f(av);
                const float z = m1 * unit_uniform(x.x0);
                const float lg = log1p_f(z);
                key = lg / wt;
                bi = (int32_t)i;
                thr = key;
                S = 0.0f;
                T = thr >= 0.0f ? INFINITY : ln_f(unit_uniform(x.x1)) / thr;
                ++nt;
                drew = true;
            }
        }
        if (a.rvs_share && __ballot(drew) != 0) take_shared_threshold(thr, T, S, wave_max(thr));
    }
    wave_argmax(key, bi);
    trig = (uint32_t)wave_sum_u64(nt);
    if (!(key > -INFINITY)) return -1;
    const uint2 e = edge_rec(a, base + bi);
    hsel = W ? __uint_as_float(e.y) : 1.0f;
    return (int32_t)e.x;
}

// rvs_step with P = 64 * V reservoir lanes (V > 1, hub rows): lane l of the wave runs the
// virtual lanes l, l + 64, ..., l + 64 (V - 1), and virtual lane vl owns items vl, vl + P,
// vl + 2P, ... (Section 3.2, parallel form).  A round reads V blocks of 64 edges at once,
// so a long row is scanned with V times the reads in flight.  Results, `trig` and `hsel`
// as for rvs_step; the lane's best virtual lane (larger index wins ties) then enters the
// wave's argmax.
template <int KIND, bool W, int V, bool EARLY>
__device__ __forceinline__ int32_t rvs_step_hub(const WalkArgs &a, const QueryDev &Q, const Mem &mem, uint32_t wid,
                                            int j, int32_t prev, int64_t base, int64_t deg, uint8_t want,
                                            const StepW &sw, uint32_t &trig, float &hsel, bool merge)
{
    constexpr int P = kWave * V;
    const int lane = lane_id();
    const uint32_t k0 = Q.key0, k1 = Q.key1;
    float key[V], thr[V], T[V], S[V];
    int32_t bi[V];
    int64_t mlo = 0;  // merge cursor in N(prev)
    // round 0: virtual lane vl keys neighbour vl, k = u^(1/w~) kept as log(u) / w~
    uint2 e0[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int64_t l = lane + kWave * v;
        e0[v] = l < deg ? edge_rec(a, base + l) : make_uint2(0u, 0u);
    }
    float kmax = -INFINITY;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int64_t l = lane + kWave * v;
        const bool memv = merge && merge_member_t<EARLY>(mem, (int32_t)e0[v].x, l < deg, mlo);
        key[v] = -INFINITY;
        bi[v] = -1;
        T[v] = 0.5f;  // holds the threshold draw until lkg is known
        if (l < deg) {
            const float wt = merge ? weight_of_member<KIND, W>(e0[v], j, prev, memv, sw)
                                   : edge_weight<KIND, W>(a, Q, base + l, e0[v], j, prev, mem, want, sw);
            const U4 x = philox(wid, (uint32_t)j, (uint32_t)l, 1u, k0, k1);
            key[v] = wt > 0.0f ? ln_f(unit_uniform(x.x0)) / wt : -INFINITY;
            T[v] = unit_uniform(x.x1);
            bi[v] = (int32_t)l;
        }
        kmax = fmaxf(kmax, key[v]);
    }
    const float lkg = wave_max(kmax);
#pragma unroll
    for (int v = 0; v < V; ++v) {
        thr[v] = lkg;
        T[v] = (lkg == -INFINITY) ? 0.0f : (lkg >= 0.0f ? INFINITY : ln_f(T[v]) / lkg);
        S[v] = 0.0f;
    }
    uint32_t nt = 0;
    // scan: a key is drawn only where a virtual lane's running weight passes its skip
    // threshold T = log(r) / log(k_thr)
    for (int64_t i0 = P; i0 < deg; i0 += P) {
        bool drew = false;
        uint2 ei[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int64_t i = i0 + lane + kWave * v;
            ei[v] = i < deg ? edge_rec(a, base + i) : make_uint2(0u, 0u);
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int64_t i = i0 + lane + kWave * v;
            const bool memi = merge && merge_member_t<EARLY>(mem, (int32_t)ei[v].x, i < deg, mlo);
            if (i < deg) {
                const float wt = merge ? weight_of_member<KIND, W>(ei[v], j, prev, memi, sw)
                                       : edge_weight<KIND, W>(a, Q, base + i, ei[v], j, prev, mem, want, sw);
                S[v] = S[v] + wt;
                if (S[v] > T[v]) {
                    // key conditioned to beat thr: log u' = log1p(expm1(w~ * thr) * V)
                    const U4 x = philox(wid, (uint32_t)j, (uint32_t)i, 1u, k0, k1);
                    const float av = wt * thr[v];
                    const float m1 = expm1_f(av);
                    const float z = m1 * unit_uniform(x.x0);
                    const float lg = log1p_f(z);
                    key[v] = lg / wt;
                    bi[v] = (int32_t)i;
                    thr[v] = key[v];
                    S[v] = 0.0f;
                    T[v] = thr[v] >= 0.0f ? INFINITY : ln_f(unit_uniform(x.x1)) / thr[v];
                    ++nt;
                    drew = true;
                }
            }
        }
        if (a.rvs_share && __ballot(drew) != 0) {
            float tm = thr[0];
#pragma unroll
            for (int v = 1; v < V; ++v) tm = fmaxf(tm, thr[v]);
            const float g = wave_max(tm);
#pragma unroll
            for (int v = 0; v < V; ++v) take_shared_threshold(thr[v], T[v], S[v], g);
        }
    }
    float key0 = key[0];
    int32_t bi0 = bi[0];
#pragma unroll
    for (int v = 1; v < V; ++v)
        if (key[v] > key0 || (key[v] == key0 && bi[v] > bi0)) {
            key0 = key[v];
            bi0 = bi[v];
        }
    float &keyb = key0;
    int32_t &bib = bi0;
    wave_argmax(keyb, bib);
    trig = (uint32_t)wave_sum_u64(nt);
    if (!(keyb > -INFINITY)) return -1;
    const uint2 e = edge_rec(a, base + bib);
    hsel = W ? __uint_as_float(e.y) : 1.0f;
    return (int32_t)e.x;
}

// eRVS for up to 64/G steps at once, one G-lane group per step, for rows of at most G
// neighbours.  Such a step is decided by round 0 alone (every neighbour gets its key,
// there is nothing to scan), so the result equals the one-wave eRVS bit for bit.
// Takes its steps from `pool` (lanes in trial order of the ballot) and returns true
// for the lanes that were served, with the next vertex (or -1) in `res` and the h of
// the chosen edge in `hres`.
template <int KIND, bool W, bool BATCH>
__device__ __forceinline__ bool rvs_group_pass(const WalkArgs &a, int G, uint64_t &pool, int32_t q, int32_t wid,
                                               int32_t j, int32_t prev, int64_t base, int32_t deg, int64_t pbase,
                                               int32_t pdeg, int32_t &res, float &hres)
{
    const int lane = lane_id();
    const int g = lane / G, r = lane % G;
    int src_of_group = -1, my_slot = -1;
    for (int s = 0; s < kWave / G; ++s) {
        int src = -1;
        if (pool != 0) {
            src = __ffsll((unsigned long long)pool) - 1;
            pool &= pool - 1;
        }
        if (g == s) src_of_group = src;
        if (lane == src) my_slot = s;
    }
    // every lane takes part in every shuffle: a step's owner may sit in a group that
    // serves nothing this pass, and a lane reading from an inactive lane gets garbage
    const int sl = src_of_group < 0 ? lane : src_of_group;
    const int32_t s_q = BATCH ? __shfl(q, sl, kWave) : 0;
    const uint32_t s_wid = (uint32_t)__shfl(wid, sl, kWave);
    const int32_t s_j = __shfl(j, sl, kWave);
    const int32_t s_prev = __shfl(prev, sl, kWave);
    const int64_t s_base = __shfl((long long)base, sl, kWave);
    const int32_t deg_of_src = __shfl(deg, sl, kWave);
    const int64_t s_pbase = __shfl((long long)pbase, sl, kWave);
    const int32_t s_pdeg = __shfl(pdeg, sl, kWave);
    const int32_t s_deg = src_of_group < 0 ? 0 : deg_of_src;
    float key = -INFINITY;
    int32_t bi = -1;
    if (r < s_deg) {
        const QueryDev &Q = query<BATCH>(a, s_q);
        const int64_t k = s_base + r;
        const uint8_t want = (KIND == kMetaPath) ? Q.schema[s_j % Q.schema_len] : (uint8_t)0;
        const Mem m = {a.col + s_pbase, s_pdeg, false, false};
        const StepW sw = step_weights<KIND>(Q, s_deg, s_pdeg);
        const float wt = edge_weight<KIND, W>(a, Q, k, edge_rec(a, k), s_j, s_prev, m, want, sw);
        const U4 x = philox(s_wid, (uint32_t)s_j, (uint32_t)r, 1u, Q.key0, Q.key1);
        key = wt > 0.0f ? ln_f(unit_uniform(x.x0)) / wt : -INFINITY;
        bi = r;
    }
    for (int o = G / 2; o > 0; o >>= 1) {
        const float k2 = __shfl_xor(key, o, kWave);
        const int32_t i2 = __shfl_xor(bi, o, kWave);
        if (k2 > key || (k2 == key && i2 > bi)) {
            key = k2;
            bi = i2;
        }
    }
    uint2 e = make_uint2(0xffffffffu, 0u);
    if (key > -INFINITY) e = edge_rec(a, s_base + bi);
    const int from = my_slot >= 0 ? my_slot * G : lane;
    const int32_t got = __shfl((int32_t)e.x, from, kWave);
    const uint32_t got_h = (uint32_t)__shfl((int32_t)e.y, from, kWave);
    if (my_slot >= 0) {
        res = got;
        hres = W ? __uint_as_float(got_h) : 1.0f;
    }
    return my_slot >= 0;
}

// Adds a wave's counters to the device totals and clears them.
__device__ __forceinline__ void flush_stats(const WalkArgs &a, uint32_t (&cnt)[kStBytes], uint64_t &bytes)
{
    const int lane = lane_id();
#pragma unroll
    for (int c = 0; c < kStBytes; ++c) {
        const uint64_t v = wave_sum_u64(cnt[c]);
        if (lane == 0 && v != 0) atomicAdd(&a.stats[c], (unsigned long long)v);
        cnt[c] = 0;
    }
    const uint64_t b = wave_sum_u64(bytes);
    if (lane == 0 && b != 0) atomicAdd(&a.stats[kStBytes], (unsigned long long)b);
    bytes = 0;
}

// BATCH: walkers of many queries (each with its own logic constants, length, seed,
// starts and outputs) share one launch; walker i of a query draws from that query's
// seed with counter (i, step, draw, tag), exactly as in a launch of its own.
// MB: the member board of plan.bound = 2 (Node2Vec, second-order PageRank); a variant of
// its own so that the lane state it needs costs the other plans no registers.
// STATS: the launch accumulates the device counters (a.stats non-null); without them the
// per-lane counts are dead code and their registers go to the walk.
// HV: virtual lanes per lane of eRVS on rows of degree >= hub_deg (P = 64 * HV there); a
// variant of its own so that the extra lane state costs the other plans no registers.
// RO: the launch samples every step by eRVS (FW_RVS_ONLY): the eRJS code is left out, and
// the eRVS merge loads each block of N(prev) ahead of the round's items (merge_member_early)
template <int KIND, bool W, bool BATCH, bool MB, bool STATS, int HV = 1, bool RO = false>
__global__ void __launch_bounds__(kBlock, (STATS || HV > 1) ? kMinWavesCounted
                                                          : (BATCH ? kMinWavesBatch : (RO ? kMinWavesRvsOnly : kMinWaves)))
walk_kernel(WalkArgs a)
{
    extern __shared__ int32_t lds_all[];
    // this wave's four slots of 64 vertex records (the first and second proposal's
    // candidate kept and alias taken), then its N(prev) staging area
    // (its offset is uniform over the wave; readfirstlane keeps it in a scalar register)
    uint4 *nvstage = reinterpret_cast<uint4 *>(lds_all) +
                     __builtin_amdgcn_readfirstlane((uint32_t)(threadIdx.x / kWave) * 4 * kWave);
    int32_t *lds = lds_all + (RO ? 0 : kWavesPerBlock * 4 * kWave * 4) + (threadIdx.x / kWave) * a.lds_cap;
    const int lane = lane_id();
    const uint64_t below = lanes_below(lane);

    int mode = kIdle;
    int32_t q = 0;     // query of the lane's walker
    int32_t wid = -1;  // walker index within its query (n < 2^31)
    int32_t cur = 0, prev = -1, j = 0, nxt = -1;
    int64_t base = 0, pbase = 0;
    int32_t deg = 0, pdeg = 0;  // degrees (nv < 2^31)
    int32_t trials = 0;
    int32_t stop_j = 0;  // resumable walks: suspend when j reaches this step
    bool fell_back = false;
    float B = 0.0f;
    float area = 0.0f;  // eRJS proposal board: deg * B (uniform) or B * h_SUM (h-proportional), plus E
    // the board's return column [0, bE) and member region [bE, bZ) of U * area; the
    // member board's h_MAX for the member test; mb: the step uses the member board
    float bE = 0.0f, bZ = 0.0f, hmx = 1.0f;
    bool mb = false;
    // h of the edge prev -> cur, and of the edge the current step takes; on a symmetric
    // graph the first is also h(cur, prev), the return edge's property weight
    float hlast = 1.0f, hnext = 1.0f;
    // path slots held back so that they go out together: from a 16-byte-aligned slot up to
    // four (one 16-byte store), from an 8-byte-aligned one two; npend slots ending at slot j
    // are held in p0, p1, p2
    int32_t p0 = 0, p1 = 0, p2 = 0, npend = 0;
    // vertex record of the next step's vertex when the accepted proposal's record carried it
    uint4 nvrec = make_uint4(0u, 0u, 0u, 0u);
    bool have_nv = false;
    // per-lane counters (32-bit counts, 64-bit bytes), flushed before a count could wrap
    uint32_t st[kStBytes];
#pragma unroll
    for (int c = 0; c < kStBytes; ++c) st[c] = 0;
    uint64_t st_bytes = 0;
    bool exhausted = false;

    for (;;) {
        if (STATS && __ballot((st[kStTrials] | st[kStTriggers] | st[kStSteps]) > 0x40000000u) != 0)
            flush_stats(a, st, st_bytes);

        // 1. hand walkers to idle lanes: one atomic per wave
        const uint64_t idle = __ballot(mode == kIdle);
        if (idle != 0 && !exhausted) {
            const int leader = __ffsll((unsigned long long)idle) - 1;
            const int cnt = __popcll(idle);
            unsigned long long first = 0;
            if (lane == leader) first = atomicAdd(a.queue, (unsigned long long)cnt);
            first = (unsigned long long)bcast_i64((int64_t)first, leader);
            if ((int64_t)first + cnt >= a.n) exhausted = true;
            if (mode == kIdle) {
                const int64_t w = (int64_t)first + __popcll(idle & below);
                if (w < a.n) {
                    const int32_t wq = BATCH ? query_of(a, w) : 0;
                    const QueryDev &Q = query<BATCH>(a, wq);
                    const int64_t local = w - Q.first;
                    int32_t *row = Q.paths + local * ((int64_t)Q.L + 1);
                    const int32_t pj = (BATCH && Q.prog) ? Q.prog[local] : 0;
                    if (pj > 0) {
                        // resume a walk suspended after pj steps: cur and prev are the last
                        // two slots it wrote, and prev's row is N(prev)
                        q = wq;
                        wid = (int32_t)local;
                        j = pj;
                        cur = row[pj];
                        prev = row[pj - 1];
                        const uint4 pr = a.vrec[prev];
                        pbase = row_start(a, pr, prev);
                        pdeg = (int32_t)pr.y;
                        hlast = 1.0f;
                        if (KIND == kNode2Vec && W && a.bound != 0) {
                            const int64_t pos = sorted_find(a.col + pbase, pdeg, cur);
                            if (pos >= 0) hlast = __uint_as_float(edge_rec(a, pbase + pos).y);
                        }
                        stop_j = pj + a.tick_steps;
                        st_bytes += 4 + 8 + 16;
                        mode = kSetup;
                    } else if (pj == 0) {
                        const int32_t s = Q.starts[local];
                        row[0] = s;
                        st_bytes += 12 + 4 * (uint64_t)Q.L;
                        if (s < 0 || (int64_t)s >= a.nv) {
                            atomicOr(a.err, 1);
                            for (int r = 1; r <= Q.L; ++r) row[r] = -1;
                            Q.lengths[local] = 0;
                            if (BATCH && Q.prog) {
                                Q.prog[local] = kDone;
                                atomicAdd(Q.done, 1);
                            }
                        } else {
                            q = wq;
                            wid = (int32_t)local;
                            cur = s;
                            prev = -1;
                            hlast = 1.0f;
                            j = 0;
                            stop_j = a.tick_steps;
                            mode = kSetup;
                        }
                    }
                }
            }
        }
        if (__ballot(mode != kIdle) == 0) {
            if (exhausted) break;
            continue;
        }

        // 2. step set-up: row of cur, bound B, strategy (Section 4.1)
        if (mode == kSetup) {
            const QueryDev &Q = query<BATCH>(a, q);
            const bool use_nv = have_nv;
            have_nv = false;
            if (j == Q.L) {
                Q.lengths[wid] = j;
                if (BATCH && Q.prog) {
                    Q.prog[wid] = kDone;
                    atomicAdd(Q.done, 1);
                }
                mode = kIdle;
                wid = -1;
            } else if (BATCH && Q.prog && j == stop_j) {
                if (npend > 0) {  // the resumed walker reads slots j - 1 and j
                    flush_path(Q.paths + (int64_t)wid * ((int64_t)Q.L + 1) + (j + 1 - npend), npend, p0, p1, p2);
                    npend = 0;
                }
                Q.prog[wid] = j;  // suspend until the next launch
                mode = kIdle;
                wid = -1;
            } else {
                const uint4 r = use_nv ? nvrec : a.vrec[cur];
                base = row_start(a, r, cur);
                deg = (int32_t)r.y;
                st_bytes += 16;
                if (deg == 0) {
                    nxt = -1;
                    mode = kAdv;
                } else if (KIND == kMetaPath && a.proposal == 2) {
                    // label-conditioned proposals: the wanted label's group of the row, whose
                    // one proposal is the sample (an eRJS cost of one trial against deg for
                    // eRVS in Eq. (runtime)); an empty group ends the walk
                    const int32_t wl = (int32_t)Q.schema[j % Q.schema_len];
                    int64_t g0 = 0, g1 = 0;
                    if (wl < a.nlab) {
                        g0 = a.lrow[(int64_t)cur * a.nlab + wl];
                        g1 = a.lrow[(int64_t)cur * a.nlab + wl + 1];
                    }
                    st_bytes += 8;
                    if (g1 == g0) {
                        nxt = -1;
                        mode = kAdv;
                    } else {
                        pbase = g0;  // MetaPath has no N(prev): these hold the group
                        pdeg = (int32_t)(g1 - g0);
                        bool rjs;
                        if (RO) {
                            rjs = false;
                        } else if (a.strategy == kRjsOnly) {
                            rjs = true;
                        } else if (a.strategy == kRandomSelect) {
                            const U4 x = philox((uint32_t)wid, (uint32_t)j, 0u, 4u, Q.key0, Q.key1);
                            rjs = unit_uniform(x.x0) < 0.5f;
                        } else if (a.strategy == kDegreeSelect) {
                            rjs = deg >= a.d_lo;
                        } else if (a.strategy == kRvsOnly) {
                            rjs = false;
                        } else {
                            rjs = deg >= a.d_lo && a.rho < (float)deg;  // a tie goes to eRVS
                        }
                        fell_back = false;
                        B = 1.0f;
                        area = 1.0f;
                        bE = 0.0f;
                        bZ = 0.0f;
                        mb = false;
                        hmx = 1.0f;
                        mode = rjs ? kRjs : kRvs;
                        trials = 0;
                    }
                } else {
                    bool rjs = false;
                    fell_back = false;
                    if (!RO && a.strategy != kRvsOnly) {
                        float wmax = (j == 0) ? Q.wmax0 : Q.wmax1;
                        float wavg = (j == 0) ? Q.wavg0 : Q.wavg1;
                        if (KIND == kSecondPR && j > 0) {
                            // max and mean over the two branches of Eq. (2ndpr) at this step
                            const StepW sw = step_weights<KIND>(Q, deg, pdeg);
                            wmax = fmaxf(sw.mem, sw.oth);
                            wavg = (sw.mem + sw.oth) / 2.0f;
                        }
                        const float hm = W ? __uint_as_float(r.z) : 1.0f;
                        const float hs = W ? __uint_as_float(r.w) : (float)deg;
                        // get_weight_max: max(w) * h_MAX; the split bound's column height
                        // leaves the return weight 1/p out; h-proportional proposals bound
                        // w alone
                        const bool split = KIND == kNode2Vec && a.bound != 0 && j > 0;
                        const bool hprop = W && a.proposal != 0;
                        const float hB = hprop ? 1.0f : hm;
                        B = split ? Q.hi_w * hB : wmax * hB;
                        const float E = split ? fmaxf(0.0f, Q.inv_p * hlast - (hprop ? B * hlast : B)) : 0.0f;
                        area = hprop ? B * hs + E : (float)deg * B + E;
                        bE = E;
                        bZ = E;
                        mb = false;
                        hmx = hm;
                        // member board: regular columns at the lower weight w_oth take every
                        // proposal, a region of area (w_mem - w_oth) * h_MAX * d(v') adds the
                        // members' excess, the return edge keeps a column for its own; used
                        // when its area is the smaller
                        if (MB && uses_membership(KIND) && j > 0 && pdeg > 0) {
                            const StepW sw = step_weights<KIND>(Q, deg, pdeg);
                            if (sw.mem > sw.oth) {
                                const float areg = hprop ? sw.oth * hs : ((float)deg * sw.oth) * hm;
                                const float Rm = ((sw.mem - sw.oth) * hm) * (float)pdeg;
                                const float Em = KIND == kNode2Vec
                                                     ? fmaxf(0.0f, Q.inv_p * hlast - sw.oth * (W ? hlast : 1.0f))
                                                     : 0.0f;
                                const float am = (areg + Rm) + Em;
                                if (am < area) {
                                    mb = true;
                                    area = am;
                                    bE = Em;
                                    bZ = Em + Rm;
                                    B = hprop ? sw.oth : sw.oth * hm;
                                }
                            }
                        }
                        if (a.strategy == kRjsOnly) {
                            rjs = true;
                            st_bytes += W ? 4 : 0;
                        } else if (a.strategy == kRandomSelect) {
                            // comparison policy: a fair coin from the walker's own stream
                            const U4 x = philox((uint32_t)wid, (uint32_t)j, 0u, 4u, Q.key0, Q.key1);
                            rjs = unit_uniform(x.x0) < 0.5f;
                            st_bytes += W ? 4 : 0;
                        } else if (a.strategy == kDegreeSelect) {
                            rjs = deg >= a.d_lo;  // comparison policy: eRJS at high degree
                            st_bytes += W ? 4 : 0;
                        } else {
                            st_bytes += W ? 8 : 0;
                            // Eq. (runtime) with get_weight_sum = mean(w) * h_SUM; with the
                            // split board or h-proportional proposals the eRJS cost is
                            // area / S per step against deg for eRVS
                            if (split || hprop || (MB && mb)) {
                                rjs = deg >= a.d_lo && (a.rho * area) < ((float)deg * (wavg * hs));
                            } else {
                                rjs = deg >= a.d_lo && (a.rho * B) < (wavg * hs);
                            }
                        }
                        // h-proportional proposals need some positive h: else eRVS
                        if (rjs && hprop && !(hs > 0.0f)) {
                            rjs = false;
                            fell_back = true;
                        }
                    }
                    mode = rjs ? kRjs : kRvs;
                    trials = 0;
                }
            }
        }

        // 3. eRJS trials inside the lane (Section 3.3): propose uniformly, accept if
        //    U * B < w~; the membership search runs only when the bounds of w~ leave
        //    the test open
        if (!RO && mode == kRjs) {
            const QueryDev &Q = query<BATCH>(a, q);
            const uint8_t want = (KIND == kMetaPath) ? Q.schema[j % Q.schema_len] : (uint8_t)0;
            // issue the loads of the next kRjsBatch proposals together, then decide them
            // in trial order; the first accepted trial is the sample, exactly as if the
            // trials ran one by one
            // split bound: a trial first picks the return edge's extra column (height
            // E) with probability E / (deg * B + E); such a trial reads no edge
            // h-proportional proposals: a record of the row's alias table gives the slot
            // and its alias; the coin is the fraction of the index draw
            // member board: a trial in the member region proposes a neighbour x of prev
            // (the index draw over d(v')); the entry (cur, x) and its h come from the edge
            // index or a search of cur's row
            // label-conditioned proposals (MetaPath): pbase and pdeg hold the wanted label's
            // group of the row; its records sit in lprop at their grouped positions
            const bool lab = KIND == kMetaPath && a.proposal == 2;
            const bool hprop = (W && a.proposal != 0) || lab;
            const int64_t pb = lab ? pbase : base;
            const int32_t pn = lab ? pdeg : deg;
            const uint4 *precs = lab ? a.lprop : a.prop;
            const bool split = KIND == kNode2Vec && a.bound != 0 && j > 0;
            const float E = MB ? bE : (split ? fmaxf(0.0f, Q.inv_p * hlast - (hprop ? B * hlast : B)) : 0.0f);
            uint32_t ux[kRjsBatch];
            uint32_t rsel[kRjsBatch];  // h-proportional: 2 (offset in the row) + (alias taken)
            uint2 ee[kRjsBatch];
            uint8_t ll[kRjsBatch];
            bool ol[kRjsBatch], mr[kRjsBatch];
            const uint32_t k0 = Q.key0, k1 = Q.key1;
            const StepW sw = step_weights<KIND>(Q, deg, pdeg);
            // a trial whose acceptance its uniforms already decide (the return column; an
            // h-proportional proposal whose test value lies below every weight the proposed
            // edge can have) makes the later proposals of the batch unnecessary: their draws
            // and loads are skipped (the decision loop stops at that trial)
            const float wsure = lab ? INFINITY
                                    : (!uses_membership(KIND) || !hprop)
                                          ? -1.0f
                                          : (j == 0 ? 1.0f : fminf(sw.ret, (MB && mb) ? sw.oth : sw.lo));
            bool sure = false;
            // the batch's first two proposals (those most often accepted) also copy their
            // two candidates' vertex records into this wave's LDS slots, in the same
            // request as the rest of the record (LDS DMA: no registers): an accepted
            // candidate's record is then read from LDS.  A line read again after its
            // first read has returned is mostly gone from L2 already (random reads turn
            // it over faster than one round trip), so a later read costs a DRAM request.
            bool nv0_ok = false;
#pragma unroll
            for (int r = 0; r < kRjsBatch; ++r) {
                if (sure) {
                    ol[r] = mr[r] = false;
                    ux[r] = 0u;
                    rsel[r] = 0u;
                    ee[r] = make_uint2(0u, 0u);
                    ll[r] = 0;
                    continue;
                }
                const U4 x = philox((uint32_t)wid, (uint32_t)j, (uint32_t)(trials + r), 0u, k0, k1);
                const int64_t k = pb + scaled_index(x.x0, x.x1, pn);
                const float z = unit_uniform(x.x3) * area;
                ol[r] = E > 0.0f && z < E;
                mr[r] = MB && uses_membership(KIND) && mb && !ol[r] && z < bZ;
                ux[r] = x.x2;
                rsel[r] = 0u;
                if (ol[r]) {
                    ee[r] = make_uint2((uint32_t)prev, 0u);
                    ll[r] = 0;
                } else if (mr[r]) {
                    ee[r] = make_uint2((uint32_t)a.col[pbase + scaled_index(x.x0, x.x1, pdeg)], 0u);
                    ll[r] = 0;
                } else if (hprop) {
                    const uint32_t f = scaled_fraction_hi(x.x0, x.x1, pn);
                    const uint4 *rec = precs + kPropU4 * k;
                    if (r < 2) {
                        __builtin_amdgcn_global_load_lds(rec + 2, lds_ptr(nvstage + 2 * r * kWave), 16, 0, 0);
                        __builtin_amdgcn_global_load_lds(rec + 3, lds_ptr(nvstage + (2 * r + 1) * kWave), 16, 0, 0);
                        if (r == 0) nv0_ok = true;
                    }
                    const uint4 r0 = rec[0], r1 = rec[1];
                    const bool keep = f < r1.x;
                    rsel[r] = ((uint32_t)(k - pb) << 1) | (keep ? 0u : 1u);
                    ee[r] = keep ? make_uint2(r0.x, r0.y) : make_uint2(r0.z, r0.w);
                    ll[r] = (KIND == kMetaPath) ? (uint8_t)(keep ? r1.y : r1.y >> 8) : (uint8_t)0;
                } else {
                    ee[r] = edge_rec(a, k);
                    ll[r] = (KIND == kMetaPath) ? a.label[k] : (uint8_t)0;
                }
                sure = ol[r] || (!mr[r] && unit_uniform(x.x2) * B < wsure);
            }
            // decide proposals in order; the batch shifts down one slot per trial so the
            // decision code appears once
#pragma unroll 1
            for (int r = 0; r < kRjsBatch; ++r) {
                const int32_t u = (int32_t)ee[0].x;
                const float hv = W ? __uint_as_float(ee[0].y) : 1.0f;
                const float hw = hprop ? 1.0f : hv;  // the test is on w~ (uniform) or w (h-proportional)
                const float y = unit_uniform(ux[0]) * B;
                float hsel = ol[0] ? hlast : hv;  // symmetric h: h(cur, prev) = h(prev, cur)
                bool acc = false;
                // a test left open by the bounds of w~ looks (lv, u) up once: in N(prev)
                // for the membership test, in N(cur) with its h for a member trial
                bool look = false;
                if (ol[0]) {
                    acc = true;  // the extra column belongs to the return edge
                } else if (MB && uses_membership(KIND) && mr[0]) {
                    // member region: keep x = u when it is a neighbour of cur (not prev),
                    // with probability h(cur, x) / h_MAX.  Bytes: x, a search of cur's row
                    // and h(cur, x)
                    st_bytes += 4 + 4 * (uint64_t)probes(deg) + (W ? 4 : 0);
                    look = u != prev;
                } else if (MB && uses_membership(KIND) && mb) {
                    // regular columns of the member board: every proposal at w_oth, the
                    // return edge at min(w_ret, w_oth)
                    acc = y < (u == prev ? fminf(sw.ret, sw.oth) : sw.oth) * hw;
                } else if (uses_membership(KIND)) {
                    if (j == 0) {
                        acc = y < hw;
                    } else if (u == prev) {
                        acc = y < sw.ret * hw;
                    } else {
                        const float lo = sw.lo * hw, hi = sw.hi * hw;
                        acc = y < lo;
                        look = !acc && y < hi;
                    }
                } else {
                    acc = y < (ll[0] == want ? hw : 0.0f);
                }
                if (uses_membership(KIND) && look) {
                    const bool mem_trial = MB && mr[0];
                    const int32_t lv = mem_trial ? cur : prev;
                    float hx = 1.0f;
                    bool found;
                    if (a.mtab) {
                        found = MB ? index_probe<true>(a.mtab, a.mtab_mask, lv, u, &hx) >= 0
                                   : index_contains(a.mtab, a.mtab_mask, lv, u);
                    } else {
                        const int64_t rb = mem_trial ? base : pbase;
                        const int32_t pos = sorted_find_interp(a.col + rb, mem_trial ? deg : pdeg, u, (int32_t)a.nv);
                        found = pos >= 0;
                        if (MB && found && W) hx = __uint_as_float(edge_rec(a, rb + pos).y);
                    }
                    if (mem_trial) {
                        hsel = W ? hx : 1.0f;
                        acc = found && unit_uniform(ux[0]) * hmx < hsel;
                    } else {
                        acc = y < (found ? sw.mem * hw : sw.oth * hw);
                    }
                }
                ++trials;
                st[kStTrials] += 1;
                // algorithmic bytes of a proposal: the proposed edge (col, h, label), the
                // alias slot's threshold and second candidate (h-proportional), and, on a
                // board whose acceptance depends on u in N(prev), a binary search of N(prev)
                // on every trial, whether or not this lane needed it
                if (STATS && !ol[0] && !mr[0])
                    st_bytes += (uint64_t)a.item_bytes + (hprop ? 12 : 0) +
                                ((uses_membership(KIND) && j > 0 && !(MB && mb)) ? 4 * (uint64_t)probes(pdeg) : 0);
                if (lab && !(hv > 0.0f)) {
                    // a proposal of weight 0 from a label group: the group's weights are all
                    // 0, so no neighbour has positive weight and the walk ends
                    nxt = -1;
                    mode = kAdv;
                    break;
                }
                if (acc) {
                    nxt = u;
                    hnext = hsel;
                    if (hprop && !ol[0] && !mr[0]) {
                        // the record's line holds the accepted candidate's vertex record
                        nvrec = (r < 2 && nv0_ok)
                                    ? nvstage[(2 * r + (rsel[0] & 1u)) * kWave + lane]
                                    : precs[kPropU4 * (pb + (int64_t)(rsel[0] >> 1)) + 2 + (rsel[0] & 1u)];
                        have_nv = true;
                    }
                    mode = kAdv;
                    st[kStRjs] += 1;
                    break;
                }
                if (trials >= a.rjs_cap) {
                    mode = kRvs;  // exact fall-back: eRVS draws are independent of eRJS draws
                    fell_back = true;
                    break;
                }
#pragma unroll
                for (int t = 0; t + 1 < kRjsBatch; ++t) {
                    ee[t] = ee[t + 1];
                    ux[t] = ux[t + 1];
                    ll[t] = ll[t + 1];
                    ol[t] = ol[t + 1];
                    mr[t] = mr[t + 1];
                    rsel[t] = rsel[t + 1];
                }
            }
        }

        // 4. eRVS for every lane that needs it (Section 5): short rows in groups of
        //    8/16/32 lanes, several steps per pass; longer rows one at a time with the
        //    whole wave
        {
            const bool want_rvs = mode == kRvs;
            uint64_t s8 = __ballot(want_rvs && deg <= 8);
            uint64_t s16 = __ballot(want_rvs && deg > 8 && deg <= 16);
            uint64_t s32 = __ballot(want_rvs && deg > 16 && deg <= 32);
            uint64_t big = __ballot(want_rvs && deg > 32);
            if (__popcll(s8) <= 4) {
                s16 |= s8;
                s8 = 0;
            }
            if (__popcll(s16) <= 2) {
                s32 |= s16;
                s16 = 0;
            }
            // the per-step accounting is the same whichever lanes served the step
            auto served = [&](int32_t res, float hres, uint32_t trig) {
                nxt = res;
                hnext = hres;
                mode = kAdv;
                st[kStTriggers] += trig;
                uint64_t by = (uint64_t)deg * (uint64_t)a.item_bytes;
                if (uses_membership(KIND) && j > 0) {
                    const uint64_t stage = 4 * (uint64_t)pdeg;
                    const uint64_t search = 4 * (uint64_t)deg * (uint64_t)probes(pdeg);
                    by += stage < search ? stage : search;
                }
                st_bytes += by;
                if (res >= 0) st[fell_back ? kStFallback : kStRvs] += 1;
            };
            int32_t res = -1;
            float hres = 1.0f;
            for (int G = 8; G <= 32; G <<= 1) {
                uint64_t &pool = G == 8 ? s8 : (G == 16 ? s16 : s32);
                while (pool != 0)
                    if (rvs_group_pass<KIND, W, BATCH>(a, G, pool, q, wid, j, prev, base, deg, pbase, pdeg, res,
                                                       hres))
                        served(res, hres, 0);
            }
            while (big != 0) {
                const int src = __ffsll((unsigned long long)big) - 1;
                big &= big - 1;
                const int32_t s_q = BATCH ? bcast_i32(q, src) : 0;
                const uint32_t s_wid = bcast_u32((uint32_t)wid, src);
                const int32_t s_j = bcast_i32(j, src);
                const int32_t s_prev = bcast_i32(prev, src);
                const int64_t s_base = bcast_i64(base, src);
                const int32_t s_deg = bcast_i32(deg, src);
                const int64_t s_pbase = bcast_i64(pbase, src);
                const int32_t s_pdeg = bcast_i32(pdeg, src);
                const QueryDev &Q = query<BATCH>(a, s_q);
                const uint8_t want = (KIND == kMetaPath) ? Q.schema[s_j % Q.schema_len] : (uint8_t)0;
                const bool member_test = uses_membership(KIND) && s_j > 0;
                Mem m = {a.col + s_pbase, s_pdeg, false, false};
                // merge the rows when N(prev) is not much longer than the row scanned
                const bool merge = member_test && (int64_t)s_pdeg <= (int64_t)kMergeRatio * s_deg;
                // stage N(prev) in LDS for the merge (its reads become LDS reads), or for the
                // per-item searches when they would read more than the staging
                if (member_test && s_pdeg <= a.lds_cap &&
                    (merge || (int64_t)s_pdeg <= (int64_t)s_deg * probes(s_pdeg))) {
                    wave_lds_sync();
                    for (int32_t i = lane; i < s_pdeg; i += kWave) lds[i] = a.col[s_pbase + i];
                    wave_lds_sync();
                    m.p = lds;
                    m.staged = true;
                }
                uint32_t trig = 0;
                const StepW sw = step_weights<KIND>(Q, s_deg, s_pdeg);
                // P = 64 lanes, or 64 * HV on a row of degree >= hub_deg
                if (HV > 1 && a.hub_deg > 0 && s_deg >= a.hub_deg)
                    res = rvs_step_hub<KIND, W, HV, RO>(a, Q, m, s_wid, s_j, s_prev, s_base, s_deg, want, sw, trig, hres,
                                                    merge);
                else
                    res = rvs_step<KIND, W, RO>(a, Q, m, s_wid, s_j, s_prev, s_base, s_deg, want, sw, trig, hres, merge);
                if (lane == src) served(res, hres, trig);
            }
        }

        // 5. apply the step (update) and write the path
        if (mode == kAdv) {
            const QueryDev &Q = query<BATCH>(a, q);
            int32_t *row = Q.paths + (int64_t)wid * ((int64_t)Q.L + 1);
            if (nxt < 0) {
                if (npend > 0) {
                    flush_path(row + (j + 1 - npend), npend, p0, p1, p2);
                    npend = 0;
                }
                // pad with -1: single slots up to a 16-byte boundary, then 16-byte stores
                int r = j + 1;
                for (; r <= Q.L && (reinterpret_cast<uintptr_t>(row + r) & 15) != 0; ++r) row[r] = -1;
                for (; r + 3 <= Q.L; r += 4) *reinterpret_cast<int4 *>(row + r) = make_int4(-1, -1, -1, -1);
                for (; r <= Q.L; ++r) row[r] = -1;
                Q.lengths[wid] = j;
                if (BATCH && Q.prog) {
                    Q.prog[wid] = kDone;
                    atomicAdd(Q.done, 1);
                }
                st[kStEarly] += 1;
                mode = kIdle;
                wid = -1;
            } else {
                const int32_t s = j + 1;
                if (npend == 0) {
                    const uintptr_t ad = reinterpret_cast<uintptr_t>(row + s);
                    if (((ad & 15) == 0 && s + 3 <= Q.L) || ((ad & 7) == 0 && s + 1 <= Q.L)) {
                        p0 = nxt;
                        npend = 1;
                    } else {
                        row[s] = nxt;
                    }
                } else {
                    int32_t *first = row + (s - npend);
                    // the group's size follows from its first slot as when it was started
                    if ((reinterpret_cast<uintptr_t>(first) & 15) != 0 || s - npend + 3 > Q.L) {
                        *reinterpret_cast<int2 *>(first) = make_int2(p0, nxt);
                        npend = 0;
                    } else if (npend == 3) {
                        *reinterpret_cast<int4 *>(first) = make_int4(p0, p1, p2, nxt);
                        npend = 0;
                    } else {
                        if (npend == 1) p1 = nxt;
                        else p2 = nxt;
                        ++npend;
                    }
                }
                st[kStSteps] += 1;
                prev = cur;
                cur = nxt;
                hlast = hnext;
                pbase = base;
                pdeg = deg;
                ++j;
                mode = kSetup;
            }
        }
    }

    if (STATS) flush_stats(a, st, st_bytes);
}

__global__ void zero_kernel(unsigned long long *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void fill_i32_kernel(int32_t *p, int64_t n, int32_t v)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// h_MAX and h_SUM per row (Section 4.2 preprocess()), one wave per row.  The sum is
// accumulated in double, so for float32 inputs of moderate range it is exact and the
// rounding to float32 does not depend on the summation order.
__global__ void __launch_bounds__(kBlock) preprocess_kernel(const int64_t *row_ptr, const float *h, int64_t nv,
                                                            uint4 *vrec)
{
    const int lane = lane_id();
    const int64_t nw = (int64_t)gridDim.x * (kBlock / kWave);
    for (int64_t v = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; v < nv; v += nw) {
        const int64_t b = row_ptr[v], e = row_ptr[v + 1];
        float mx = 0.0f;
        double sm = 0.0;
        for (int64_t k = b + lane; k < e; k += kWave) {
            const float x = h ? h[k] : 1.0f;
            mx = x > mx ? x : mx;
            sm += (double)x;
        }
        mx = wave_max(mx);
        sm = wave_sum_f64(sm);
        if (lane == 0) vrec[v] = make_uint4((uint32_t)b, (uint32_t)(e - b), __float_as_uint(mx), __float_as_uint((float)sm));
    }
}

// Device layout: {col, h} edge records and {start, degree, -, -} vertex records.
// 8-bit property weights: h = h_scale * code, one float32 product.
__global__ void dequantize_kernel(const uint8_t *code, float h_scale, int64_t ne, float *h)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < ne; k += stride)
        h[k] = (float)code[k] * h_scale;
}

// 8-bit property weights on graphs of at most 2^24 vertices: a 4-byte edge record.
__global__ void pack8_kernel(const int32_t *col, const uint8_t *code, int64_t ne, uint32_t *erec8)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < ne; k += stride)
        erec8[k] = (uint32_t)col[k] | ((uint32_t)code[k] << 24);
}

__global__ void layout_kernel(const int64_t *row_ptr, const int32_t *col, const float *h, int64_t nv, int64_t ne,
                              uint2 *edges, uint4 *vrec, uint32_t *start_hi)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (edges)
        for (int64_t k = t0; k < ne; k += stride)
            edges[k] = make_uint2((uint32_t)col[k], __float_as_uint(h ? h[k] : 1.0f));
    for (int64_t v = t0; v < nv; v += stride) {
        const int64_t b = row_ptr[v], e = row_ptr[v + 1];
        vrec[v] = make_uint4((uint32_t)b, (uint32_t)(e - b), 0u, 0u);
        if (start_hi) start_hi[v] = (uint32_t)((uint64_t)b >> 32);
    }
}

__global__ void validate_rows_kernel(const int64_t *row_ptr, int64_t nv, int64_t ne, int *err)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= nv; v += stride) {
        bool bad = false;
        if (v == 0 && row_ptr[0] != 0) bad = true;
        if (v == nv && row_ptr[nv] != ne) bad = true;
        if (v < nv && row_ptr[v] > row_ptr[v + 1]) bad = true;
        if (bad) atomicOr(err, 1);
    }
}

__global__ void __launch_bounds__(kBlock) validate_edges_kernel(const int64_t *row_ptr, const int32_t *col,
                                                                const float *h, int64_t nv, int *err,
                                                                unsigned long long *max_deg)
{
    const int lane = lane_id();
    const int64_t nw = (int64_t)gridDim.x * (kBlock / kWave);
    unsigned long long dmax = 0;
    for (int64_t v = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; v < nv; v += nw) {
        const int64_t b = row_ptr[v], e = row_ptr[v + 1];
        dmax = (unsigned long long)(e - b) > dmax ? (unsigned long long)(e - b) : dmax;
        bool bad = false;
        for (int64_t k = b + lane; k < e; k += kWave) {
            const int32_t c = col[k];
            if (c < 0 || (int64_t)c >= nv) bad = true;
            if (k > b && col[k - 1] >= c) bad = true;
            if (h) {
                const float x = h[k];
                if (!(x >= 0.0f) || isinf(x)) bad = true;
            }
        }
        if (bad) atomicOr(err, 2);
    }
    if (lane == 0 && dmax > 0) atomicMax(max_deg, dmax);
}

// Proposal records of h-proportional eRJS: Walker's alias table of each row's h, built
// with the sweeping construction of Huebschle-Schneider and Sanders (Parallel Weighted
// Random Sampling) in exact integer arithmetic, here in its parallel form.  Row v with n
// entries: q_k = floor(h_k / h_MAX * 2^32) (double quotient, one rounding; 2^32 when the
// row has no positive h or the graph is unweighted), Q = sum q_k, entry k brings
// a_k = q_k * n units to buckets of Q units; light entries (a_k < Q) have the deficit
// Q - a_k, heavy ones the surplus a_k - Q.  With D the deficits of the light entries
// before a given one and E the surplus of the heavy entries up to a given one (both in
// index order), the sequential sweep is equivalent to:
//   * light entry i keeps a_i and takes as alias the first heavy entry j with E_j >= D_i;
//   * heavy entry j keeps Q + E_j - D(n_j), where n_j counts the light entries with
//     D_i <= E_j and D(n_j) is their total deficit (the total of all deficits, which
//     equals the last E, when n_j covers them all); unless it keeps a full Q its alias is
//     the next heavy entry.
// Sums of up to 2^31 values below 2^63 need 128 bits; everything is an integer, so the
// result does not depend on the order of any sum.  A bucket keeping K units stores the
// threshold min(floor(K * 2^32 / Q), 2^32 - 1).
//
// Pass 1 (one wave per row): Q, then each light entry's D and each heavy entry's E, the
// light entries compacted at the row's front in index order and the heavy ones at its
// back in reverse order (val: the 128-bit sum, idx: the entry's offset), and {Q, light
// count} per row.  Pass 2 (one wave per row): both merges of the two sorted sequences,
// 64 entries of each at a time, and the 64-byte record of every entry:
//   {col_k, bits(h_k), col_a, bits(h_a)}, {threshold, label_k | label_a << 8, a, 0},
//   vrec[col_k], vrec[col_a]   (a: the alias's offset in the row).
using u128 = unsigned __int128;

// The sums of a row of n entries stay below n * Q <= n^2 * 2^32 (every q_k <= 2^32): 64 bits
// hold them for rows of at most 2^15 entries, which take the 64-bit path (half the lane
// exchanges of the 128-bit one).
constexpr int64_t kAlias64Max = (int64_t)1 << 15;
// Rows longer than this are merged by alias_hub_kernel, many waves per row.
constexpr int64_t kAliasHubRow = 8192;
// Rows of at most this many entries are built by alias_small_kernel, one lane per row.
constexpr int64_t kAliasSmallRow = 16;

template <typename T>
__device__ __forceinline__ T shfl_t(T x, int src)
{
    if constexpr (sizeof(T) == 8) {
        return (T)__shfl((long long)x, src, kWave);
    } else {
        const uint64_t lo = (uint64_t)__shfl((long long)(uint64_t)x, src, kWave);
        const uint64_t hi = (uint64_t)__shfl((long long)(uint64_t)(x >> 64), src, kWave);
        return ((u128)hi << 64) | lo;
    }
}

template <typename T>
__device__ __forceinline__ T shfl_up_t(T x, int d)
{
    if constexpr (sizeof(T) == 8) {
        return (T)__shfl_up((long long)x, d, kWave);
    } else {
        const uint64_t lo = (uint64_t)__shfl_up((long long)(uint64_t)x, d, kWave);
        const uint64_t hi = (uint64_t)__shfl_up((long long)(uint64_t)(x >> 64), d, kWave);
        return ((u128)hi << 64) | lo;
    }
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan_t(T x)
{
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const T y = shfl_up_t(x, d);
        if (lane >= d) x += y;
    }
    return x;
}

// A sum as stored in `val` (16 bytes, zero-extended from 64 bits).
template <typename T>
__device__ __forceinline__ T load_t(const uint4 *p)
{
    const uint4 x = *p;
    if constexpr (sizeof(T) == 8) return ((uint64_t)x.y << 32) | (uint64_t)x.x;
    else return ((u128)x.w << 96) | ((u128)x.z << 64) | ((u128)x.y << 32) | (u128)x.x;
}

template <typename T>
__device__ __forceinline__ uint4 pack_t(T x)
{
    return make_uint4((uint32_t)x, (uint32_t)((uint64_t)x >> 32), (uint32_t)((u128)x >> 64), (uint32_t)((u128)x >> 96));
}

// q_k of the construction: h_k relative to the row maximum in 32 fractional bits.
__device__ __forceinline__ uint64_t alias_q(const float *h, int64_t k, float hmax)
{
    if (h == nullptr || !(hmax > 0.0f)) return (uint64_t)1 << 32;
    return (uint64_t)floor(((double)h[k] / (double)hmax) * 4294967296.0);
}

__device__ __forceinline__ uint32_t alias_thr(u128 keep, uint64_t Q)
{
    const u128 t = (keep << 32) / (u128)Q;
    return t >= (u128)0xFFFFFFFFu ? 0xFFFFFFFFu : (uint32_t)t;
}

// Pass 1 on row [b, b + n) with maximum hmax, sums of type T.
template <typename T>
__device__ __forceinline__ void alias_scan_row(const float *h, int64_t b, int64_t n, float hmax, uint4 *val,
                                               int32_t *idx, ulonglong2 *rowinfo_v)
{
    const int lane = lane_id();
    const uint64_t below = lanes_below(lane);
    uint64_t qs = 0;
    for (int64_t k = lane; k < n; k += kWave) qs += alias_q(h, b + k, hmax);
    const uint64_t Q = wave_sum_u64(qs);
    T dcarry = 0, ecarry = 0;
    int64_t nl = 0, nh = 0;
    for (int64_t k0 = 0; k0 < n; k0 += kWave) {
        const int64_t k = k0 + lane;
        const bool valid = k < n;
        const uint64_t a = valid ? alias_q(h, b + k, hmax) * (uint64_t)n : 0;
        const bool light = valid && a < Q, heavy = valid && a >= Q;
        const uint64_t lm = __ballot(light), hm = __ballot(heavy);
        const T d = light ? (T)(Q - a) : (T)0, e = heavy ? (T)(a - Q) : (T)0;
        const T dinc = wave_incl_scan_t(d), einc = wave_incl_scan_t(e);
        if (light) {
            const int64_t pos = b + nl + __popcll(lm & below);
            val[pos] = pack_t<T>(dcarry + dinc - d);  // deficits before this entry
            idx[pos] = (int32_t)k;
        }
        if (heavy) {
            const int64_t pos = b + n - 1 - (nh + __popcll(hm & below));
            val[pos] = pack_t<T>(ecarry + einc);  // surplus up to and including this entry
            idx[pos] = (int32_t)k;
        }
        dcarry += shfl_t(dinc, kWave - 1);
        ecarry += shfl_t(einc, kWave - 1);
        nl += __popcll(lm);
        nh += __popcll(hm);
    }
    if (lane == 0) *rowinfo_v = make_ulonglong2((unsigned long long)Q, (unsigned long long)nl);
}

__global__ void __launch_bounds__(kBlock) alias_scan_kernel(const int64_t *row_ptr, const float *h, int64_t nv,
                                                            const uint4 *vrec, const float *rmax, uint4 *val,
                                                            int32_t *idx, ulonglong2 *rowinfo)
{
    const int64_t nw = (int64_t)gridDim.x * (kBlock / kWave);
    for (int64_t v = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; v < nv; v += nw) {
        const int64_t b = row_ptr[v];
        const int64_t n = row_ptr[v + 1] - b;
        if (n <= kAliasSmallRow) continue;  // alias_small_kernel
        const float hmax = rmax ? rmax[v] : __uint_as_float(vrec[v].z);
        if (n <= kAlias64Max) alias_scan_row<uint64_t>(h, b, n, hmax, val, idx, rowinfo + v);
        else alias_scan_row<u128>(h, b, n, hmax, val, idx, rowinfo + v);
    }
}

// Index of the first of the 64 wave lanes whose x (ascending over the lanes) is >= key
// (ge) or > key (!ge); 64 when there is none.
template <typename T>
__device__ __forceinline__ int wave_bound_t(T x, T key, bool ge)
{
    int c = 0;
#pragma unroll
    for (int s = kWave / 2; s > 0; s >>= 1) {
        const T y = shfl_t(x, c + s - 1);
        if (ge ? (y < key) : (y <= key)) c += s;
    }
    // c in [0, 63]: one more test decides between c and 64
    const T y = shfl_t(x, c);
    return (ge ? (y < key) : (y <= key)) ? c + 1 : c;
}

__device__ __forceinline__ void write_record(const int32_t *col, const float *h, const uint8_t *label,
                                             const uint4 *vrec, int64_t b, int32_t k, int32_t al, uint32_t thr,
                                             uint4 *prop)
{
    const uint32_t hk = h ? __float_as_uint(h[b + k]) : __float_as_uint(1.0f);
    const uint32_t ha = h ? __float_as_uint(h[b + al]) : __float_as_uint(1.0f);
    const uint32_t lab = label ? ((uint32_t)label[b + k] | ((uint32_t)label[b + al] << 8)) : 0u;
    const int32_t ck = col[b + k], ca = col[b + al];
    uint4 *r = prop + (int64_t)kPropU4 * (b + k);
    r[0] = make_uint4((uint32_t)ck, hk, (uint32_t)ca, ha);
    r[1] = make_uint4(thr, lab, (uint32_t)al, 0u);
    r[2] = vrec[ck];
    r[3] = vrec[ca];
}

// Pass 2 on row [b, b + n) with Q and nl from pass 1, sums of type T.
template <typename T>
__device__ __forceinline__ void alias_merge_row(const int32_t *col, const float *h, const uint8_t *label,
                                                const uint4 *vrec, const uint4 *val, const int32_t *idx, int64_t b,
                                                int64_t n, uint64_t Q, int64_t nl, float hmax, uint4 *prop)
{
    const int lane = lane_id();
    constexpr T kMax = ~(T)0;
    const int64_t nh = n - nl;  // >= 1 (the caller checked)
    // heavy entry j (in index order) sits at b + n - 1 - j
    const T e_last = load_t<T>(val + b + n - nh);
    // light entries: alias = the first heavy entry whose E reaches the entry's D
    for (int64_t li = 0, hj = 0; li < nl;) {
        if (hj >= nh) {
            // unreachable in exact arithmetic (the last E equals the total deficit, so
            // every light entry finds its heavy one); kept so that the loop always ends
            // and every record stays a valid self-alias
            for (int64_t i = li + lane; i < nl; i += kWave) {
                const int32_t k = idx[b + i];
                write_record(col, h, label, vrec, b, k, k, 0xFFFFFFFFu, prop);
            }
            break;
        }
        const int64_t i = li + lane, j = hj + lane;
        const T D = i < nl ? load_t<T>(val + b + i) : kMax;
        const T E = j < nh ? load_t<T>(val + b + n - 1 - j) : kMax;
        const int32_t hix = j < nh ? idx[b + n - 1 - j] : -1;
        const int c = wave_bound_t(E, D, true);
        const bool found = i < nl && c < kWave && hj + c < nh;
        const int32_t al = __shfl(hix, c & (kWave - 1), kWave);
        const int cnt = __popcll(__ballot(found));  // a prefix of the lanes (D ascends)
        if (cnt == 0) {
            hj += kWave;
            continue;
        }
        if (found) {
            const int32_t k = idx[b + i];
            const uint64_t a = alias_q(h, b + k, hmax) * (uint64_t)n;
            write_record(col, h, label, vrec, b, k, al, alias_thr((u128)a, Q), prop);
        }
        li += cnt;
    }
    // heavy entries: keep Q + E_j - D(n_j), alias the next heavy entry unless full
    for (int64_t hj = 0, li = 0; hj < nh;) {
        const int64_t i = li + lane, j = hj + lane;
        const T D = i < nl ? load_t<T>(val + b + i) : kMax;
        const T E = j < nh ? load_t<T>(val + b + n - 1 - j) : kMax;
        const int c = wave_bound_t(D, E, false);  // light entries with D <= E_j in this block
        const bool found = j < nh && c < kWave;
        const T dn = shfl_t(D, c & (kWave - 1));
        const int cnt = __popcll(__ballot(found));  // a prefix of the lanes (E ascends)
        if (cnt == 0) {
            li += kWave;
            continue;
        }
        if (found) {
            const T spent = li + c < nl ? dn : e_last;
            const T keep = (T)Q + E - spent;
            const int32_t k = idx[b + n - 1 - j];
            const int32_t al = (keep < (T)Q && j + 1 < nh) ? idx[b + n - 2 - j] : k;
            write_record(col, h, label, vrec, b, k, al, alias_thr((u128)keep, Q), prop);
        }
        hj += cnt;
    }
}

__global__ void __launch_bounds__(kBlock) alias_merge_kernel(const int64_t *row_ptr, const int32_t *col,
                                                             const float *h, const uint8_t *label, int64_t nv,
                                                             const uint4 *vrec, const float *rmax, const uint4 *val,
                                                             const int32_t *idx, const ulonglong2 *rowinfo,
                                                             uint4 *prop)
{
    const int lane = lane_id();
    const int64_t nw = (int64_t)gridDim.x * (kBlock / kWave);
    for (int64_t v = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; v < nv; v += nw) {
        const int64_t b = row_ptr[v];
        const int64_t n = row_ptr[v + 1] - b;
        if (n <= kAliasSmallRow) continue;  // alias_small_kernel
        const ulonglong2 ri = rowinfo[v];
        const uint64_t Q = (uint64_t)ri.x;
        const int64_t nl = (int64_t)ri.y;
        if (n - nl <= 0) {  // unreachable (the a_k sum to n * Q); every record stays a valid self-alias
            for (int64_t k = lane; k < n; k += kWave)
                write_record(col, h, label, vrec, b, (int32_t)k, (int32_t)k, 0xFFFFFFFFu, prop);
            continue;
        }
        if (n > kAliasHubRow) continue;  // alias_hub_kernel
        const float hmax = rmax ? rmax[v] : __uint_as_float(vrec[v].z);
        if (n <= kAlias64Max) alias_merge_row<uint64_t>(col, h, label, vrec, val, idx, b, n, Q, nl, hmax, prop);
        else alias_merge_row<u128>(col, h, label, vrec, val, idx, b, n, Q, nl, hmax, prop);
    }
}

// Rows of 1 .. kAliasSmallRow entries, one lane per row: the sweep itself, in entry order.
// A(k) = q_k * n.  With the current heavy entry j holding residual r: each light entry i
// (A < Q) first closes the heavy entries whose residual has fallen below Q (bucket j keeps
// r, aliased to the next heavy entry, which then holds A(j') - (Q - r)), then keeps A(i)
// with j as its alias, and r loses Q - A(i); the heavy entries left at the end are closed
// the same way, a full bucket being its own alias.  This is the table the two passes
// above build for longer rows (sums here stay below 16 * 16 * 2^32).
__global__ void __launch_bounds__(256) alias_small_kernel(const int64_t *row_ptr, const int32_t *col, const float *h,
                                                          const uint8_t *label, int64_t nv, const uint4 *vrec,
                                                          const float *rmax, uint4 *prop)
{
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < nv; v += (int64_t)gridDim.x * 256) {
        const int64_t b = row_ptr[v];
        const int32_t n = (int32_t)(row_ptr[v + 1] - b);
        if (n == 0 || n > kAliasSmallRow) continue;
        const float hmax = rmax ? rmax[v] : __uint_as_float(vrec[v].z);
        uint64_t Q = 0;
        for (int32_t k = 0; k < n; ++k) Q += alias_q(h, b + k, hmax);
        auto A = [&](int32_t k) { return alias_q(h, b + k, hmax) * (uint64_t)n; };
        int32_t j = 0;
        while (A(j) < Q) ++j;  // the first heavy entry (the A sum to n * Q)
        uint64_t r = A(j);
        for (int32_t i = 0; i < n; ++i) {
            const uint64_t ai = A(i);
            if (ai >= Q) continue;
            while (r < Q) {  // a later heavy entry exists while a light entry is left
                int32_t jn = j + 1;
                while (jn < n - 1 && A(jn) < Q) ++jn;
                write_record(col, h, label, vrec, b, j, jn, alias_thr((u128)r, Q), prop);
                r = A(jn) - (Q - r);
                j = jn;
            }
            write_record(col, h, label, vrec, b, i, j, alias_thr((u128)ai, Q), prop);
            r -= Q - ai;
        }
        for (;;) {
            int32_t jn = j + 1;
            while (jn < n && A(jn) < Q) ++jn;
            write_record(col, h, label, vrec, b, j, (r < Q && jn < n) ? jn : j, alias_thr((u128)r, Q), prop);
            if (jn >= n) break;
            r = A(jn) - (Q - r);
            j = jn;
        }
    }
}

// The rows longer than kAliasHubRow, appended to `hubs` in any order (*nhub counts them).
__global__ void __launch_bounds__(256) alias_hub_list_kernel(const int64_t *row_ptr, int64_t nv, int32_t *hubs,
                                                             int *nhub)
{
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < nv; v += (int64_t)gridDim.x * 256)
        if (row_ptr[v + 1] - row_ptr[v] > kAliasHubRow) hubs[atomicAdd(nhub, 1)] = (int32_t)v;
}

// Pass 2 for the long rows, one thread per entry (blockIdx.y picks the row, the blocks of a
// row stride over its entries): the same two merges, each entry finding its partner by a
// binary search of the other sorted sequence instead of a wave walking the row, so that a
// hub row is spread over many waves.  Light entry i: alias = the first heavy entry with
// E >= D_i.  Heavy entry j: keep Q + E_j - D(first light entry with D > E_j, or the last
// E), alias the next heavy entry unless it keeps a full bucket.
__global__ void __launch_bounds__(256) alias_hub_kernel(const int64_t *row_ptr, const int32_t *col, const float *h,
                                                        const uint8_t *label, const uint4 *vrec, const float *rmax,
                                                        const uint4 *val, const int32_t *idx,
                                                        const ulonglong2 *rowinfo, const int32_t *hubs,
                                                        const int *nhub, uint4 *prop)
{
    const int nh_rows = *nhub;
    for (int hr = blockIdx.y; hr < nh_rows; hr += gridDim.y) {
        const int64_t v = hubs[hr];
        const int64_t b = row_ptr[v];
        const int64_t n = row_ptr[v + 1] - b;
        const ulonglong2 ri = rowinfo[v];
        const uint64_t Q = (uint64_t)ri.x;
        const int64_t nl = (int64_t)ri.y, nh = n - nl;
        const float hmax = rmax ? rmax[v] : __uint_as_float(vrec[v].z);
        for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) {
            if (nh <= 0) {  // unreachable (the a_k sum to n * Q); a valid self-alias
                write_record(col, h, label, vrec, b, (int32_t)t, (int32_t)t, 0xFFFFFFFFu, prop);
                continue;
            }
            if (t < nl) {
                const u128 D = load_t<u128>(val + b + t);
                int64_t lo = 0, hi = nh;  // first heavy j with E_j >= D (E_j at b + n - 1 - j, ascending in j)
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (load_t<u128>(val + b + n - 1 - mid) < D) lo = mid + 1;
                    else hi = mid;
                }
                const int32_t k = idx[b + t];
                if (lo >= nh) {  // unreachable in exact arithmetic; a valid self-alias
                    write_record(col, h, label, vrec, b, k, k, 0xFFFFFFFFu, prop);
                    continue;
                }
                const uint64_t a = alias_q(h, b + k, hmax) * (uint64_t)n;
                write_record(col, h, label, vrec, b, k, idx[b + n - 1 - lo], alias_thr((u128)a, Q), prop);
            } else {
                const int64_t j = t - nl;
                const u128 E = load_t<u128>(val + b + n - 1 - j);
                int64_t lo = 0, hi = nl;  // first light i with D_i > E (D ascending in i)
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (load_t<u128>(val + b + mid) <= E) lo = mid + 1;
                    else hi = mid;
                }
                const u128 spent = lo < nl ? load_t<u128>(val + b + lo) : load_t<u128>(val + b + n - nh);
                const u128 keep = (u128)Q + E - spent;
                const int32_t k = idx[b + n - 1 - j];
                const int32_t al = (keep < (u128)Q && j + 1 < nh) ? idx[b + n - 2 - j] : k;
                write_record(col, h, label, vrec, b, k, al, alias_thr(keep, Q), prop);
            }
        }
    }
}

// Edge index build: one wave per row, each lane inserts its entries' keys with a 64-bit
// compare-and-swap into the first free slot from the key's bucket on, then stores the
// entry's h in the slot's h part (rows are strictly ascending, so a key is inserted once).
// The table holds at least twice as many slots as keys, so every insert finds a slot
// within the scan.  tab: 16 uint64 per bucket (8 keys, then 8 h as float pairs).
__global__ void __launch_bounds__(kBlock) build_index_kernel(const int64_t *row_ptr, const int32_t *col,
                                                             const float *h, int64_t nv, unsigned long long *tab,
                                                             uint64_t mask)
{
    const int lane = lane_id();
    const int64_t nw = (int64_t)gridDim.x * (kBlock / kWave);
    for (int64_t v = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; v < nv; v += nw) {
        const int64_t b = row_ptr[v], e = row_ptr[v + 1];
        for (int64_t k = b + lane; k < e; k += kWave) {
            const unsigned long long key = edge_key((int32_t)v, col[k]);
            uint64_t bk = mix64(key) & mask;
            bool done = false;
            for (uint64_t t = 0; t <= mask && !done; ++t) {
                for (int s = 0; s < 8 && !done; ++s) {
                    unsigned long long *bucket = tab + bk * (2 * kIndexBucketU4);
                    const unsigned long long old = atomicCAS(&bucket[s], kEmptyKey, key);
                    done = old == kEmptyKey || old == key;
                    if (old == kEmptyKey) reinterpret_cast<float *>(bucket + 8)[s] = h ? h[k] : 1.0f;
                }
                bk = (bk + 1) & mask;
            }
        }
    }
}

// One wave per row v: every entry (v, u) must have the reverse entry (u, v) with the
// same h bits, else bit 4 of *err is set (one atomic per wave).
__global__ void __launch_bounds__(kBlock) check_symmetry_kernel(const int64_t *row_ptr, const int32_t *col,
                                                                const float *h, int64_t nv, int *err)
{
    const int lane = lane_id();
    const int64_t nw = (int64_t)gridDim.x * (kBlock / kWave);
    bool bad = false;
    for (int64_t v = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; v < nv; v += nw) {
        const int64_t b = row_ptr[v], e = row_ptr[v + 1];
        for (int64_t k = b + lane; k < e; k += kWave) {
            const int32_t u = col[k];
            const int64_t ub = row_ptr[u];
            const int64_t pos = sorted_find(col + ub, row_ptr[u + 1] - ub, (int32_t)v);
            if (pos < 0) bad = true;
            else if (h && __float_as_uint(h[ub + pos]) != __float_as_uint(h[k])) bad = true;
        }
    }
    if (__ballot(bad) != 0 && lane == 0) atomicOr(err, 16);
}

// Candidate nodes for the profiling kernels: candidate k is vertex k * stride (k < n), reported
// as {vertex, degree}.
__global__ void __launch_bounds__(kBlock) profile_pick_kernel(const int64_t *row_ptr, int64_t stride, int n,
                                                             int2 *out)
{
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const int64_t v = (int64_t)k * stride;
    out[k] = make_int2((int32_t)v, (int32_t)(row_ptr[v + 1] - row_ptr[v]));
}

hipError_t launch_profile_pick(const int64_t *row_ptr, int64_t stride, int n, int2 *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(profile_pick_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       row_ptr, stride, n, out);
    return hipGetLastError();
}

// Profiling kernels (Section 5, "Flexi-Runtime Profiling Kernels"): evaluate workload
// weights of sampled nodes either as eRVS does (a wave scanning a row, coalesced) or
// as eRJS does (a lane proposing random neighbours).  Their time ratio per edge is the
// EdgeCost_RJS / EdgeCost_RVS constant of Eq. (runtime).
template <int KIND, bool W>
__global__ void __launch_bounds__(kBlock) profile_rvs_kernel(WalkArgs a, const int32_t *nodes, int nsample,
                                                             int per_node, float *sink)
{
    const int lane = lane_id();
    const int nw = gridDim.x * (kBlock / kWave);
    float acc = 0.0f;
    for (int s = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; s < nsample; s += nw) {
        const int32_t v = nodes[s];
        const uint4 rv = a.vrec[v];
        const int64_t b = row_start(a, rv, v), d = (int64_t)rv.y;
        const int64_t m = d < per_node ? d : per_node;
        const int32_t prev = a.col[b];
        const uint4 rp = a.vrec[prev];
        const int64_t pb = row_start(a, rp, prev), pd = (int64_t)rp.y;
        for (int64_t i = lane; i < m; i += kWave)
            acc += edge_weight<KIND, W>(a, a.q0, b + i, edge_rec(a, b + i), 1, prev, Mem{a.col + pb, pd, false, false},
                                        a.q0.schema[0], step_weights<KIND>(a.q0, (int32_t)d, (int32_t)pd));
    }
    acc = wave_max(acc);
    if (lane == 0 && acc < 0.0f) sink[0] = acc;  // never true; keeps the loads alive
}

template <int KIND, bool W>
__global__ void __launch_bounds__(kBlock) profile_rjs_kernel(WalkArgs a, const int32_t *nodes, int nsample,
                                                             int per_node, float *sink)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    float acc = 0.0f;
    if (s < nsample) {
        const int32_t v = nodes[s];
        const uint4 rv = a.vrec[v];
        const int64_t b = row_start(a, rv, v), d = (int64_t)rv.y;
        const int32_t prev = a.col[b];
        const uint4 rp = a.vrec[prev];
        const int64_t pb = row_start(a, rp, prev), pd = (int64_t)rp.y;
        for (int t = 0; t < per_node; ++t) {
            const U4 x = philox((uint32_t)s, 0u, (uint32_t)t, 2u, a.q0.key0, a.q0.key1);
            const int64_t k = b + scaled_index(x.x0, x.x1, d);
            acc += edge_weight<KIND, W>(a, a.q0, k, edge_rec(a, k), 1, prev, Mem{a.col + pb, pd, false, true}, a.q0.schema[0],
                                        step_weights<KIND>(a.q0, (int32_t)d, (int32_t)pd));
        }
    }
    if (acc < 0.0f) sink[0] = acc;
}

// Random-read ceiling: each lane issues four independent 8-byte loads per round at
// addresses hashed from (lane, round), masked into a power-of-two array.  Its rate is the
// memory system's limit for the access pattern the walk kernel's proposals make.
__global__ void __launch_bounds__(kBlock) random_reads_kernel(const uint2 *a, uint64_t mask, int rounds,
                                                              unsigned *sink)
{
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned acc = 0;
    for (int it = 0; it < rounds; ++it) {
        uint2 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = a[mix64(t * 1315423911ull + (uint64_t)it * 64 + (uint64_t)k) & mask];
#pragma unroll
        for (int k = 0; k < 4; ++k) acc += v[k].x ^ v[k].y;
    }
    if (acc == 0x9E3779B9u) sink[0] = acc;  // keeps the loads; practically never true
}

// ---------------------------------------------------------------- launchers
hipError_t launch_random_reads(const uint2 *a, uint64_t mask, int blocks, int rounds, unsigned *sink, hipStream_t s)
{
    hipLaunchKernelGGL(random_reads_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, a, mask, rounds, sink);
    return hipGetLastError();
}

template <int KIND, bool W, bool BATCH, bool STATS, int HV>
static void launch_walk_h(const WalkArgs &a, int grid, size_t lds, hipStream_t s)
{
    if (!BATCH && a.strategy == kRvsOnly)
        hipLaunchKernelGGL((walk_kernel<KIND, W, BATCH, false, STATS, HV, !BATCH>), dim3(grid), dim3(kBlock),
                           walk_lds_bytes(a.lds_cap, true), s, a);
    else if (uses_membership(KIND) && a.bound == 2)
        hipLaunchKernelGGL((walk_kernel<KIND, W, BATCH, uses_membership(KIND), STATS, HV>), dim3(grid), dim3(kBlock),
                           lds, s, a);
    else
        hipLaunchKernelGGL((walk_kernel<KIND, W, BATCH, false, STATS, HV>), dim3(grid), dim3(kBlock), lds, s, a);
}

// hub lanes (P > 64 on long rows) are built for single-query launches only
template <int KIND, bool W, bool BATCH, bool STATS>
static void launch_walk_s(const WalkArgs &a, int grid, size_t lds, hipStream_t s)
{
    const int hv = (BATCH || a.hub_deg <= 0) ? 1 : a.hub_v;
    if (!BATCH && hv == 4) launch_walk_h<KIND, W, BATCH, STATS, (BATCH ? 1 : 4)>(a, grid, lds, s);
    else if (!BATCH && hv == 2) launch_walk_h<KIND, W, BATCH, STATS, (BATCH ? 1 : 2)>(a, grid, lds, s);
    else launch_walk_h<KIND, W, BATCH, STATS, 1>(a, grid, lds, s);
}

template <int KIND, bool W, bool BATCH>
static hipError_t launch_walk_t(const WalkArgs &a, int grid, hipStream_t s)
{
    const size_t lds = walk_lds_bytes(a.lds_cap);
    if (a.stats != nullptr) launch_walk_s<KIND, W, BATCH, true>(a, grid, lds, s);
    else launch_walk_s<KIND, W, BATCH, false>(a, grid, lds, s);
    return hipGetLastError();
}

template <bool BATCH>
static hipError_t launch_walk_b(const WalkArgs &a, int kind, bool weighted, int grid, hipStream_t s)
{
    if (kind == kNode2Vec) return weighted ? launch_walk_t<kNode2Vec, true, BATCH>(a, grid, s)
                                           : launch_walk_t<kNode2Vec, false, BATCH>(a, grid, s);
    if (kind == kSecondPR) return weighted ? launch_walk_t<kSecondPR, true, BATCH>(a, grid, s)
                                           : launch_walk_t<kSecondPR, false, BATCH>(a, grid, s);
    return weighted ? launch_walk_t<kMetaPath, true, BATCH>(a, grid, s)
                    : launch_walk_t<kMetaPath, false, BATCH>(a, grid, s);
}

hipError_t launch_walk(const WalkArgs &a, int kind, bool weighted, bool batch, int grid, hipStream_t s)
{
    return batch ? launch_walk_b<true>(a, kind, weighted, grid, s) : launch_walk_b<false>(a, kind, weighted, grid, s);
}

template <int KIND, bool W, bool BATCH, bool RO>
static int occupancy_blocks(int lds_cap)
{
    int nb = 0;
    const size_t lds = walk_lds_bytes(lds_cap, RO);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, walk_kernel<KIND, W, BATCH, false, false, 1, RO>, kBlock,
                                                     lds) != hipSuccess)
        nb = 1;
    return nb > 0 ? nb : 1;
}

template <bool BATCH, bool RO>
static int occupancy_b(int kind, bool weighted, int lds_cap)
{
    if (kind == kNode2Vec) return weighted ? occupancy_blocks<kNode2Vec, true, BATCH, RO>(lds_cap)
                                           : occupancy_blocks<kNode2Vec, false, BATCH, RO>(lds_cap);
    if (kind == kSecondPR) return weighted ? occupancy_blocks<kSecondPR, true, BATCH, RO>(lds_cap)
                                           : occupancy_blocks<kSecondPR, false, BATCH, RO>(lds_cap);
    return weighted ? occupancy_blocks<kMetaPath, true, BATCH, RO>(lds_cap)
                    : occupancy_blocks<kMetaPath, false, BATCH, RO>(lds_cap);
}

int walk_grid(int kind, bool weighted, bool batch, int lds_cap, int64_t n, bool rvs_only)
{
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (cus <= 0) cus = 1;
    const int nb = batch ? occupancy_b<true, false>(kind, weighted, lds_cap)
                         : (rvs_only ? occupancy_b<false, true>(kind, weighted, lds_cap)
                                     : occupancy_b<false, false>(kind, weighted, lds_cap));
    int64_t grid = (int64_t)nb * cus;
    const int64_t need = (n + kBlock - 1) / kBlock;
    if (grid > need) grid = need;
    return (int)(grid > 0 ? grid : 1);
}

hipError_t launch_zero(unsigned long long *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(zero_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_preprocess(const int64_t *row_ptr, const float *h, int64_t nv, uint4 *vrec, hipStream_t s)
{
    int64_t blocks = (nv + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(preprocess_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, row_ptr, h, nv, vrec);
    return hipGetLastError();
}

hipError_t launch_layout(const int64_t *row_ptr, const int32_t *col, const float *h, int64_t nv, int64_t ne,
                         uint2 *edges, uint4 *vrec, uint32_t *start_hi, hipStream_t s)
{
    int64_t work = ne > nv ? ne : nv;
    int64_t blocks = (work + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(layout_kernel, dim3((unsigned)blocks), dim3(256), 0, s, row_ptr, col, h, nv, ne, edges, vrec,
                       start_hi);
    return hipGetLastError();
}

hipError_t launch_validate_rows(const int64_t *row_ptr, int64_t nv, int64_t ne, int *err, hipStream_t s)
{
    int64_t blocks = (nv + 1 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(validate_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, s, row_ptr, nv, ne, err);
    return hipGetLastError();
}

hipError_t launch_validate_edges(const int64_t *row_ptr, const int32_t *col, const float *h, int64_t nv,
                                 int *err, unsigned long long *max_deg, hipStream_t s)
{
    int64_t blocks = (nv + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(validate_edges_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, row_ptr, col, h, nv, err,
                       max_deg);
    return hipGetLastError();
}

__global__ void export_alias_kernel(const uint4 *prop, int64_t ne, uint32_t *thr, int32_t *alias)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < ne; k += stride) {
        const uint4 r1 = prop[(int64_t)kPropU4 * k + 1];
        thr[k] = r1.x;
        alias[k] = (int32_t)r1.z;
    }
}

hipError_t launch_export_alias(const uint4 *prop, int64_t ne, uint32_t *thr, int32_t *alias, hipStream_t s)
{
    if (ne <= 0) return hipSuccess;
    int64_t blocks = (ne + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(export_alias_kernel, dim3((unsigned)blocks), dim3(256), 0, s, prop, ne, thr, alias);
    return hipGetLastError();
}

hipError_t launch_build_alias(const int64_t *row_ptr, const int32_t *col, const float *h, const uint8_t *label,
                              int64_t nv, const uint4 *vrec, const float *rmax, uint4 *val, int32_t *idx,
                              ulonglong2 *rowinfo, int32_t *hubs, int *nhub, uint4 *prop, hipStream_t s)
{
    int64_t blocks = (nv + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(alias_scan_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, row_ptr, h, nv, vrec, rmax, val,
                       idx, rowinfo);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(alias_merge_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, row_ptr, col, h, label, nv,
                       vrec, rmax, val, idx, rowinfo, prop);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the short rows, one lane each
    int64_t sb = (nv + 255) / 256;
    if (sb > 65536) sb = 65536;
    if (sb < 1) sb = 1;
    hipLaunchKernelGGL(alias_small_kernel, dim3((unsigned)sb), dim3(256), 0, s, row_ptr, col, h, label, nv, vrec, rmax,
                       prop);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the long rows: listed, then one thread per entry
    if ((e = hipMemsetAsync(nhub, 0, sizeof(int), s)) != hipSuccess) return e;
    int64_t lb = (nv + 255) / 256;
    if (lb > 4096) lb = 4096;
    if (lb < 1) lb = 1;
    hipLaunchKernelGGL(alias_hub_list_kernel, dim3((unsigned)lb), dim3(256), 0, s, row_ptr, nv, hubs, nhub);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(alias_hub_kernel, dim3(64, 1024), dim3(256), 0, s, row_ptr, col, h, label, vrec, rmax, val, idx,
                       rowinfo, hubs, nhub, prop);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) label_max_kernel(const uint8_t *label, int64_t ne, int *out)
{
    int m = 0;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < ne; k += (int64_t)gridDim.x * 256)
        m = max(m, (int)label[k]);
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, kWave));
    if (lane_id() == 0 && m > 0) atomicMax(out, m);
}

hipError_t launch_label_max(const uint8_t *label, int64_t ne, int *out, hipStream_t s)
{
    if (ne <= 0) return hipSuccess;
    int64_t blocks = (ne + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(label_max_kernel, dim3((unsigned)blocks), dim3(256), 0, s, label, ne, out);
    return hipGetLastError();
}

// Label groups, one wave per row: pass 1 counts each label's entries and takes its h maximum
// (a ballot and a wave maximum per label and 64-entry chunk), pass 2 scatters the entries in
// row order to their group's next positions (rank = earlier entries of the same label).
__global__ void __launch_bounds__(kBlock) label_group_kernel(const int64_t *row_ptr, const int32_t *col,
                                                             const float *h, const uint8_t *label, int64_t nv,
                                                             int nlab, int64_t *lrow, float *gmax, int32_t *vcol,
                                                             float *vh, uint8_t *vlab)
{
    const int lane = lane_id();
    const uint64_t below = lanes_below(lane);
    const int64_t nw = (int64_t)gridDim.x * (kBlock / kWave);
    for (int64_t v = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; v < nv; v += nw) {
        const int64_t b = row_ptr[v], n = row_ptr[v + 1] - b;
        int64_t pos[kMaxLabels];
        float mx[kMaxLabels];
#pragma unroll
        for (int l = 0; l < kMaxLabels; ++l) {
            pos[l] = 0;
            mx[l] = 0.0f;
        }
        for (int64_t k0 = 0; k0 < n; k0 += kWave) {
            const int64_t k = k0 + lane;
            const int lab = k < n ? (int)label[b + k] : -1;
            const float hv = k < n ? (h ? h[b + k] : 1.0f) : 0.0f;
#pragma unroll
            for (int l = 0; l < kMaxLabels; ++l) {
                if (l < nlab) {
                    const uint64_t m = __ballot(lab == l);
                    pos[l] += __popcll(m);
                    if (m != 0) mx[l] = fmaxf(mx[l], wave_max(lab == l ? hv : 0.0f));
                }
            }
        }
        int64_t start = b;
#pragma unroll
        for (int l = 0; l < kMaxLabels; ++l) {
            if (l < nlab) {
                if (lane == 0) {
                    lrow[v * nlab + l] = start;
                    gmax[v * nlab + l] = mx[l];
                }
                const int64_t c = pos[l];
                pos[l] = start;
                start += c;
            }
        }
        for (int64_t k0 = 0; k0 < n; k0 += kWave) {
            const int64_t k = k0 + lane;
            const int lab = k < n ? (int)label[b + k] : -1;
#pragma unroll
            for (int l = 0; l < kMaxLabels; ++l) {
                if (l < nlab) {
                    const uint64_t m = __ballot(lab == l);
                    if (lab == l) {
                        const int64_t p = pos[l] + __popcll(m & below);
                        vcol[p] = col[b + k];
                        if (vh) vh[p] = h[b + k];
                        vlab[p] = (uint8_t)l;
                    }
                    pos[l] += __popcll(m);
                }
            }
        }
    }
}

hipError_t launch_label_groups(const int64_t *row_ptr, const int32_t *col, const float *h, const uint8_t *label,
                               int64_t nv, int nlab, int64_t *lrow, float *gmax, int32_t *vcol, float *vh,
                               uint8_t *vlab, hipStream_t s)
{
    if (nv <= 0) return hipSuccess;
    int64_t blocks = (nv + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(label_group_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, row_ptr, col, h, label, nv,
                       nlab, lrow, gmax, vcol, vh, vlab);
    return hipGetLastError();
}

hipError_t launch_dequantize(const uint8_t *code, float h_scale, int64_t ne, float *h, hipStream_t s)
{
    if (ne <= 0) return hipSuccess;
    int64_t blocks = (ne + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(dequantize_kernel, dim3((unsigned)blocks), dim3(256), 0, s, code, h_scale, ne, h);
    return hipGetLastError();
}

hipError_t launch_pack8(const int32_t *col, const uint8_t *code, int64_t ne, uint32_t *erec8, hipStream_t s)
{
    if (ne <= 0) return hipSuccess;
    int64_t blocks = (ne + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(pack8_kernel, dim3((unsigned)blocks), dim3(256), 0, s, col, code, ne, erec8);
    return hipGetLastError();
}

hipError_t launch_build_index(const int64_t *row_ptr, const int32_t *col, const float *h, int64_t nv,
                              unsigned long long *tab, uint64_t mask, hipStream_t s)
{
    int64_t blocks = (nv + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(build_index_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, row_ptr, col, h, nv, tab,
                       mask);
    return hipGetLastError();
}

hipError_t launch_check_symmetry(const int64_t *row_ptr, const int32_t *col, const float *h, int64_t nv, int *err,
                                 hipStream_t s)
{
    int64_t blocks = (nv + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(check_symmetry_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, row_ptr, col, h, nv, err);
    return hipGetLastError();
}

template <int KIND, bool W>
static hipError_t launch_profile_t(const WalkArgs &a, bool rjs_style, const int32_t *nodes, int nsample,
                                   int per_node, float *sink, hipStream_t s)
{
    if (rjs_style) {
        hipLaunchKernelGGL((profile_rjs_kernel<KIND, W>), dim3((nsample + kBlock - 1) / kBlock), dim3(kBlock), 0,
                           s, a, nodes, nsample, per_node, sink);
    } else {
        int blocks = (nsample + kWavesPerBlock - 1) / kWavesPerBlock;
        hipLaunchKernelGGL((profile_rvs_kernel<KIND, W>), dim3(blocks), dim3(kBlock), 0, s, a, nodes, nsample,
                           per_node, sink);
    }
    return hipGetLastError();
}

hipError_t launch_profile(const WalkArgs &a, int kind, bool weighted, bool rjs_style, const int32_t *nodes,
                          int nsample, int per_node, float *sink, hipStream_t s)
{
    if (kind == kNode2Vec)
        return weighted ? launch_profile_t<kNode2Vec, true>(a, rjs_style, nodes, nsample, per_node, sink, s)
                        : launch_profile_t<kNode2Vec, false>(a, rjs_style, nodes, nsample, per_node, sink, s);
    if (kind == kSecondPR)
        return weighted ? launch_profile_t<kSecondPR, true>(a, rjs_style, nodes, nsample, per_node, sink, s)
                        : launch_profile_t<kSecondPR, false>(a, rjs_style, nodes, nsample, per_node, sink, s);
    return weighted ? launch_profile_t<kMetaPath, true>(a, rjs_style, nodes, nsample, per_node, sink, s)
                    : launch_profile_t<kMetaPath, false>(a, rjs_style, nodes, nsample, per_node, sink, s);
}

}  // namespace fw
