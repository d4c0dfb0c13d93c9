/*
 * flexiwalk.h -- C ABI of the MI355X (gfx950) dynamic random-walk sampler.
 *
 * The library runs the per-step transition sampling of FlexiWalker (arXiv 2512.00705):
 * at every step each walker evaluates runtime-dependent weights w~ = w * h over the
 * neighbours of its current vertex (Section 2.1, Eq. prob) and draws the next vertex
 * with exponential-key reservoir sampling plus jumps (eRVS, Section 3.2, Algorithm 1,
 * Eq. jump) or bounded rejection sampling (eRJS, Section 3.3), picked per step by the
 * first-order cost model (Section 4.1, Eq. runtime).  All work runs in HIP kernels.
 *
 * Conventions for every call:
 *   - return value: FW_OK (0) or an fw_status code; fw_last_error() gives a message
 *     (thread-local, valid until the next call on the same thread);
 *   - "device pointer": memory on the current HIP device (e.g. a torch tensor's
 *     data_ptr()); "host pointer": ordinary process memory;
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Kernel
 *     launches are asynchronous on that stream; argument errors are returned before
 *     anything is enqueued.
 *   - A graph may be used by many fw_walk calls, but calls that share one graph must
 *     be ordered on one stream (they share the graph's work counter).
 */
#ifndef FLEXIWALK_H
#define FLEXIWALK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fw_status {
    FW_OK = 0,
    FW_E_INVALID = 1, /* bad argument or malformed input; nothing was changed */
    FW_E_NOMEM = 2,   /* device allocation failed; nothing was allocated */
    FW_E_DEVICE = 3,  /* a HIP runtime call failed */
    FW_E_STATE = 4,   /* object not ready (e.g. graph not preprocessed) */
    FW_E_BUSY = 5     /* the server's waiting queue is full; retry later */
} fw_status;

/* Sampling strategy per step: the cost model of Section 4.1 (AUTO), the single-kernel
 * modes of the ablation, and the two selection policies the evaluation compares the cost
 * model with (sensitivity on selection strategy): a fair coin per step drawn from the
 * walker's stream (Philox counter (walker, step, 0, 4), eRJS iff U(x0) < 1/2), and eRVS
 * below the degree plan.d_lo (1K in the paper) with eRJS at or above it. */
enum { FW_AUTO = 0, FW_RVS_ONLY = 1, FW_RJS_ONLY = 2, FW_RANDOM_SELECT = 4, FW_DEGREE_SELECT = 5 };

/* Walk logics (Section 2.1). */
enum { FW_NODE2VEC = 1, FW_METAPATH = 2, FW_SECOND_PR = 3 };

#define FW_MAX_SCHEMA 64
#define FW_NSTATS 8

/* CSR graph handed to fw_graph_create.  Row v holds the neighbours N(v) in
 * col[row_ptr[v] .. row_ptr[v+1]), strictly ascending (Node2Vec tests membership in
 * N(prev) by binary search).  h: per-edge property weights h(v,u) >= 0, finite (NULL:
 * unweighted, h = 1).  label: per-edge labels for MetaPath (NULL if unused).  All
 * arrays are host pointers when on_device == 0, device pointers when 1. */
typedef struct fw_csr {
    int64_t nv, ne;
    const int64_t *row_ptr; /* nv + 1 entries, row_ptr[0] = 0, row_ptr[nv] = ne */
    const int32_t *col;     /* ne entries in [0, nv) */
    const float *h;         /* ne entries or NULL */
    const uint8_t *label;   /* ne entries or NULL */
    int32_t on_device;
    /* 8-bit property weights (the low-precision edge weights of Section 7): ne codes or
     * NULL.  When given, h must be NULL and h(v,u) = h_scale * code, one float32 product
     * (round to nearest); the walk then reads a 4-byte record {col in bits 0..23, code in
     * bits 24..31} per edge when nv <= 2^24 (else the usual 8-byte {col, h} record of the
     * dequantised weight).  Samples depend only on the dequantised weights. */
    const uint8_t *h8;
    float h_scale;          /* finite, > 0 when h8 is given; ignored otherwise */
} fw_csr;

typedef struct fw_graph fw_graph; /* opaque, library-owned device copy of a graph */

/* Walk logic (value type).
 * FW_NODE2VEC (Eq. node2vec): w = 1/p if u is the previous vertex, 1 if u is a
 *   neighbour of the previous vertex, 1/q otherwise; p, q are the paper's a, b.  The
 *   first step of a walk has no previous vertex and uses w = 1.
 * FW_METAPATH (Section 2.1): w = 1 if the label of edge (v,u) equals
 *   schema[j mod schema_len] at step j, else 0; a walk ends when no neighbour has
 *   positive weight.
 * FW_SECOND_PR (Eq. 2ndpr): with max_d = max(d(v), d(v')), w = ((1 - gamma)/d(v) +
 *   gamma/d(v')) * max_d if u is a neighbour of the previous vertex v', else
 *   ((1 - gamma)/d(v)) * max_d (the return to v' included); evaluated in float32 in that
 *   order.  The first step has no previous vertex and uses w = 1.
 * weighted: 1 uses w~ = w * h, 0 uses w~ = w. */
typedef struct fw_logic {
    int32_t kind;
    int32_t weighted;
    float p, q;
    float gamma;
    int32_t schema_len;
    uint8_t schema[FW_MAX_SCHEMA];
} fw_logic;

/* Plan.  rho, d_lo and rjs_cap change which kernel samples a step and therefore the
 * random stream (never the distribution); the remaining fields change speed only.
 *   rho      EdgeCost_RJS / EdgeCost_RVS of Eq. (runtime), > 0
 *   d_lo     steps at vertices of degree < d_lo always use eRVS (0 disables)
 *   rjs_cap  eRJS trials before an exact fall-back to eRVS, >= 1
 *   lanes    eRVS lanes P per step below hub_deg; must be 64 (one wavefront)
 *   hub_deg  rows of at least this degree are scanned by eRVS with hub_lanes lanes (0: never)
 *   hub_lanes eRVS lanes P for those rows: 64, 128 or 256 (the wave runs P / 64 virtual lanes
 *            per lane, so a round reads P / 64 blocks of 64 edges at once); P changes which
 *            items share a skip threshold and so the random stream, never the distribution;
 *            fw_walk only: fw_batch_create, fw_batch_run_noalloc and fw_server_create
 *            return FW_E_INVALID for hub_deg > 0 with hub_lanes != 64
 *   rvs_share 0 or 1 (changes the stream, never the distribution).  0: each eRVS lane
 *            keeps its own threshold after the shared round-0 maximum (Section 3.2,
 *            parallel description).  1 (an extension): after every scan round in which
 *            some lane drew a key, each lane below the largest threshold thr_g takes it
 *            and rescales its remaining skip, T' = ((T - S) * thr) / thr_g in float32
 *            (the remaining skip is exponential with rate -thr; scaled, it is the skip
 *            of thr_g), S' = 0; a lane with no threshold yet (-inf) keeps T = 0, and
 *            thr_g >= 0 makes T' = +inf.  Keys below thr_g cannot win, so only fewer
 *            keys are drawn.  A round is P items (hub_lanes on hub rows).
 *   lds_cap  int32 entries of N(prev) staged in LDS per wavefront, 0..8192 (0: never stage)
 *   grid     persistent blocks (0 = fill the device)
 *   bound    eRJS bound (changes the stream, never the distribution):
 *            0  max(w) * h_MAX of Section 3.3;
 *            1  Node2Vec split bound, an extension of Section 3.3 (any bound that
 *               dominates every w~ keeps eRJS exact): columns of height
 *               max(1, 1/q) * h_MAX plus one extra column holding the return edge's
 *               excess (1/p) * h(cur, prev) - that height, taken with probability
 *               excess / (deg * height + excess) per trial.  Needs a graph whose
 *               reverse edges exist with equal h (fw_graph_info reports it); MetaPath
 *               ignores it.  The cost model then compares rho * (deg * height +
 *               excess) with deg * S^.
 *            2  member board (extension of Section 3.3), Node2Vec with q > 1 and
 *               second-order PageRank with gamma > 0, where members of N(prev) weigh
 *               w_mem above everyone else's w_oth: regular columns at w_oth take every
 *               proposal (no membership test; the return edge at min(w_ret, w_oth)),
 *               the return edge keeps an extra column (w_ret - w_oth) * h(v, prev), and
 *               a member region of area (w_mem - w_oth) * h_MAX * d(prev) proposes a
 *               neighbour x of prev uniformly and keeps it when (v, x) is an edge, with
 *               probability h(v, x) / h_MAX (the edge index, else a search of v's row,
 *               finds it).  Per step the smaller of this board and bound 1's (Node2Vec)
 *               or bound 0's is used; the cost model compares rho * (its area) with
 *               deg * S^.  Node2Vec needs a symmetric graph as for 1.
 *   proposal eRJS proposal distribution (changes the stream, never the distribution):
 *            0  uniform over N(v) (Section 3.3), tested as U * B < w~;
 *            1  proportional to the static weight h(v,u) through per-row alias tables
 *               (fw_graph_build_alias), tested as U * W < w with W >= every workload
 *               weight: the mass of u is h * w / (W * sum h), proportional to w~, and the
 *               expected trials drop from deg * B / S to W * h_SUM / S.  Applies to
 *               weighted logics; a row whose h are all zero goes to eRVS.  With
 *               bound = 1 the return edge's extra column is (1/p - W) * h(v, prev) wide.
 *            2  as 1 for Node2Vec and second-order PageRank; MetaPath proposes from the
 *               wanted label's group of the row through its own alias table
 *               (fw_graph_build_label_alias; an extension of Section 3.3, not in the
 *               paper): the MetaPath weight is h on the schema's label and 0 elsewhere,
 *               so that proposal is the sample (one trial).  An empty group, or one whose
 *               h are all 0, ends the walk.  The cost model weighs that one trial against
 *               the eRVS scan: eRJS iff deg >= d_lo and rho < deg.
 *            The cost model compares rho * (board area) with deg * S^ for 1 (and bound 1). */
typedef struct fw_plan {
    float rho;
    int32_t d_lo;
    int32_t rjs_cap;
    int32_t lanes;
    int32_t lds_cap;
    int32_t grid;
    int32_t bound;
    int32_t proposal;
    int32_t hub_deg;
    int32_t hub_lanes;
    int32_t rvs_share;
} fw_plan;

/* Counters accumulated by fw_walk into a device array of FW_NSTATS uint64 values:
 *   0 steps taken, 1 steps sampled by eRJS, 2 steps sampled by eRVS, 3 eRJS steps that
 *   reached rjs_cap and fell back to eRVS, 4 eRJS trials, 5 eRVS jump events (keys drawn
 *   after round 0), 6 walks that ended before L steps, 7 algorithmic bytes (the bytes
 *   the method itself must move: row pointers, bounds, scanned or proposed edges,
 *   membership probes, start/path/length I/O). */

/* Copy a CSR graph into library-owned device memory (Section 2.1 graph G with N(v),
 * d(v), h, labels); nv < 2^30.  Validates row_ptr (monotone, row_ptr[0] = 0, row_ptr[nv] = ne), col
 * (in range, strictly ascending per row) and h (finite, >= 0); on failure returns
 * FW_E_INVALID and allocates nothing.  Device-side inputs are validated on the device
 * before the call returns (synchronous).  *out is set only on FW_OK. */
int fw_graph_create(const fw_csr *g, fw_graph **out);

/* Free a graph and its device memory.  NULL is accepted.  The caller must ensure no
 * work that uses the graph is still running. */
int fw_graph_destroy(fw_graph *g);

/* Per-node preprocessing (Section 4.2, preprocess()): h_MAX[v] = max h over N(v) and
 * h_SUM[v] = sum of h over N(v) accumulated in double precision and rounded once to
 * float32 (0 for an empty row).  Asynchronous on `stream`; idempotent.  Must run before
 * fw_walk with a weighted logic. */
int fw_graph_preprocess(fw_graph *g, void *stream);

/* Copy h_MAX and h_SUM (nv floats each, host pointers) back to the host; synchronous. */
int fw_graph_export_aux(const fw_graph *g, float *hmax, float *hsum);

/* Build the edge index: an exact hash map of the entries (v, u) to h(v, u) (128-byte
 * buckets of eight 64-bit keys and their eight float h, at most half full; 32 bytes of
 * device memory per entry, rounded up to a power-of-two bucket count).  The membership
 * test u in N(prev) of an eRJS proposal (Node2Vec, second-order PageRank) then reads one
 * bucket instead of searching prev's sorted row, and so does a member-board trial's
 * lookup of (cur, x) with its h; eRVS steps keep searching the row, which all lanes of the
 * step share.  Samples and counts of eRJS trials do not change (the algorithmic-byte
 * counter charges 8 bytes per membership test and 12 per member lookup instead of a
 * binary search's).  Asynchronous on `stream`; idempotent.  Walks, batches and servers created
 * afterwards use it; build it before creating batches or servers.  Returns FW_E_NOMEM if
 * the table cannot be allocated (the graph stays usable without it). */
int fw_graph_build_index(fw_graph *g, void *stream);

/* Build the proposal records of h-proportional eRJS (plan.proposal = 1): per CSR entry k
 * of row v, 64 bytes {col[k], h[k], col[a], h[a]}, {threshold, labels of k and a, a, 0} and
 * the vertex records (row start, degree, h_MAX, h_SUM) of col[k] and col[a], where a (an
 * offset in the row) and the threshold form Walker's alias table of the row's h.  The
 * table is built with the sweeping construction (Huebschle-Schneider and Sanders,
 * "Parallel Weighted Random Sampling") in exact integer arithmetic: q_k = floor(h_k /
 * h_MAX * 2^32) (2^32 for every entry when the graph is unweighted or the row has no
 * positive h), buckets of Q = sum q_k units, entry k bringing q_k * deg units; a bucket
 * keeping K units has threshold min(floor(K * 2^32 / Q), 2^32 - 1), so entry k is proposed
 * with probability q_k / Q.  The result does not depend on how the construction is
 * scheduled (one wave per row here, a sequential sweep in a reference).  A proposal takes
 * slot floor(R * deg / 2^64) of a 64-bit draw R and keeps it when the high 32 bits of the
 * fraction lie below the threshold, else takes a.  A record sits in one DRAM line.  Runs
 * fw_graph_preprocess first if it has not run.  Device memory: 64 bytes per entry, plus
 * 20 bytes per entry and 16 per vertex of scratch while building.  Synchronous;
 * idempotent.  Walks, batches and servers created afterwards can use it. */
int fw_graph_build_alias(fw_graph *g, void *stream);

/* Label groups for label-conditioned MetaPath proposals (plan.proposal = 2): the entries
 * of each row taken in (label, row position) order, so that the entries of label l form
 * group (v, l), and one alias table per group over its h (the construction of
 * fw_graph_build_alias, with the group's h maximum; 1 per entry on an unweighted graph).
 * Device memory: a 64-byte record per entry in grouped order, as fw_graph_build_alias
 * writes them (the alias field holds the slot within the group), and 8 bytes per (vertex,
 * label) for the group starts; while building, 45 bytes per entry and 20 per (vertex,
 * label) of scratch.  Needs edge labels, all below 16 (FW_E_INVALID otherwise; FW_E_STATE
 * without labels).  Runs fw_graph_preprocess first if it has not run.  Synchronous;
 * idempotent. */
int fw_graph_build_label_alias(fw_graph *g, void *stream);

/* Copy the alias tables behind the proposal records to the host (ne entries each, host
 * pointers): thr[k] = the keep threshold of slot k, alias[k] = the row offset of its alias.
 * For replaying the sample stream outside the library.  Synchronous; FW_E_STATE before
 * fw_graph_build_alias. */
int fw_graph_export_alias(const fw_graph *g, uint32_t *thr, int32_t *alias);

/* Roofline calibration (not part of the method): time random 8-byte reads from a device
 * array of `bytes` (a power of two >= 1 MiB), 2^20 lanes each issuing four independent
 * loads per round, and store the best rate in *reads_per_s.  Each such read moves one
 * 128-byte line from HBM, so this is the ceiling for the walk kernel's proposal, vertex
 * and membership reads.  Allocates and frees its array; synchronous on `stream`. */
int fw_calibrate_random_reads(int64_t bytes, double *reads_per_s, void *stream);

/* Sizes of a graph: vertices, edges, maximum degree, and 1 if every edge (v, u) has a
 * reverse edge (u, v) with the same h (checked on the device by fw_graph_create), else 0
 * (any pointer may be NULL). */
int fw_graph_info(const fw_graph *g, int64_t *nv, int64_t *ne, int64_t *max_deg, int32_t *symmetric);

/* Build a Node2Vec logic; p, q finite and > 0. */
int fw_logic_node2vec(float p, float q, int32_t weighted, fw_logic *out);

/* Build a MetaPath logic from `m` labels (1 <= m <= FW_MAX_SCHEMA, host pointer). */
int fw_logic_metapath(const uint8_t *schema, int32_t m, int32_t weighted, fw_logic *out);

/* Build a second-order PageRank logic; 0 <= gamma <= 1. */
int fw_logic_second_pr(float gamma, int32_t weighted, fw_logic *out);

/* Default plan: rho = 8, d_lo = 0, rjs_cap = 1024, lanes = 64, hub_deg = 0 (every row at
 * 64 lanes), hub_lanes = 64, lds_cap and grid chosen by the library. */
int fw_plan_default(fw_plan *out);

/* Profiling kernels of Section 5: time weight evaluation of a sample of the nodes (the
 * non-isolated ones among up to 32768 evenly spaced vertex ids, at most 16384) with
 * eRJS-style random proposals and with eRVS-style coalesced scans on this graph and
 * logic, and set out->rho to the per-edge cost ratio EdgeCost_RJS / EdgeCost_RVS of
 * Eq. (runtime); the other fields come from fw_plan_default.  Synchronous on `stream`;
 * the graph must be preprocessed for a weighted logic. */
int fw_plan_profile(fw_graph *g, const fw_logic *logic, fw_plan *out, void *stream);

/* fw_plan_profile, then a measured search: short seeded sample walks (up to 2^20 walkers,
 * 16 steps, AUTO) are timed for rho scaled by 1/16 .. 4 around the profiled value (with
 * each eRJS bound: the split bound and the member board too for Node2Vec on a symmetric
 * graph, the member board for second-order PageRank; and each
 * proposal: h-proportional too for a weighted logic once fw_graph_build_alias ran, and
 * label-conditioned for MetaPath once fw_graph_build_label_alias ran), then for the
 * degree gate d_lo in {0, 8, 32, 128}, the LDS budget for N(prev) (lds_cap in
 * {256, 512, 1024, 2048, 4096}), the eRJS trial cap
 * rjs_cap in {16, 64, 256, 1024, 4096}, the lanes' shared eRVS threshold (rvs_share,
 * taken only when 2 % faster), the eRVS lanes on long rows (hub_lanes 128 or
 * 256 from hub_deg 1024 or 8192; fw_plan_autotune only, never for a mix) and the
 * persistent grid (the occupancy limit, half of it, twice it); the fastest plan is
 * returned.  Every candidate
 * samples the same distribution; only the choice of kernel per step, and so the random
 * stream, differs.  Allocates temporary device memory; synchronous on `stream`. */
int fw_plan_autotune(fw_graph *g, const fw_logic *logic, fw_plan *out, void *stream);

/* fw_plan_autotune for a mix of logics, such as the queries of a batch or the requests a
 * server takes (Section 5, dynamic query scheduling: one plan serves every query of a
 * launch).  rho is profiled on logics[0]; each candidate plan is timed on every logic
 * (each with an equal share of the sample walkers, at least 2^18): when the logics share
 * kind and weighting (one batch can hold them) as one batch of one query per logic, in
 * the batched kernel that batches and the server run; otherwise as one fw_walk launch per
 * logic, scored by the sum.
 * Only bounds every logic accepts are tried.  logics: host array of n_logics values,
 * 1 <= n_logics <= 64.  Same allocation and synchronisation as fw_plan_autotune;
 * fw_plan_autotune(g, lg, out, s) equals fw_plan_autotune_mix(g, lg, 1, out, s). */
int fw_plan_autotune_mix(fw_graph *g, const fw_logic *logics, int32_t n_logics, fw_plan *out, void *stream);

/* Run n walks of at most L steps (Section 5 runtime kernel with dynamic query
 * scheduling).
 *   starts  device pointer, n int32 start vertices
 *   paths   device pointer, n * (L + 1) int32: paths[i*(L+1)] = starts[i], slot k holds
 *           the vertex after k steps, -1 after the walk ended
 *   lengths device pointer, n int32: steps taken (0..L)
 *   stats   device pointer to FW_NSTATS uint64 counters that are ADDED to, or NULL
 * Walker i draws its random numbers from Philox4x32-10 keyed by `seed` with counter
 * (i, step, draw, tag), so results do not depend on the launch shape.  0 <= L < 2^20,
 * 0 <= n < 2^31.  A start vertex outside [0, nv) gives that walker length 0 and marks the
 * graph's error flag, reported by fw_graph_check.  Asynchronous on `stream`. */
int fw_walk(fw_graph *g, const fw_logic *logic, const fw_plan *plan, int32_t strategy,
            const int32_t *starts, int64_t n, int32_t L, uint64_t seed, int32_t *paths,
            int32_t *lengths, uint64_t *stats, void *stream);

/* One query of a batch: `n` walkers of at most L steps with the given logic and seed.
 * Its start vertices are starts[start_off .. start_off + n), its paths occupy
 * paths[out_off .. out_off + n*(L+1)) in the fw_walk layout and its lengths
 * lengths[len_off .. len_off + n).  Walker i of the query uses Philox counter (i, step,
 * draw, tag) under key `seed`, so its walk is the same as in fw_walk of that query alone. */
typedef struct fw_query {
    fw_logic logic;
    int64_t n;
    int32_t L;
    uint64_t seed;
    int64_t start_off;
    int64_t out_off;
    int64_t len_off;
} fw_query;

typedef struct fw_batch fw_batch; /* opaque: a query table resident on the device */

/* Prepare a batch of nq queries (host array) over graph g for one persistent launch
 * (Section 5 runtime kernel; dynamic scheduling over the walkers of all queries).  All
 * queries share the logic kind and weighting (mixed kinds go in separate batches).
 * starts, paths and lengths are device pointers owned by the caller and bound to the
 * batch, holding starts_len, paths_len and lengths_len int32 elements: every query's
 * blocks must lie inside them (FW_E_INVALID otherwise), must not overlap, and the arrays
 * must stay valid while the batch is used.  Copies the query table to the device
 * (synchronous); does not launch.  The plan and strategy apply to all queries. */
int fw_batch_create(fw_graph *g, const fw_query *queries, int64_t nq, const fw_plan *plan, int32_t strategy,
                    const int32_t *starts, int64_t starts_len, int32_t *paths, int64_t paths_len,
                    int32_t *lengths, int64_t lengths_len, fw_batch **out);

/* Run every query of the batch in one launch on `stream` (asynchronous).  Allocates
 * nothing and issues no memset or host synchronisation, so it can be captured into a HIP
 * graph.  stats: device pointer to FW_NSTATS uint64 counters added to, or NULL.
 * Launches of one batch must be ordered on one stream (they share its walker counter). */
int fw_batch_launch(fw_batch *b, uint64_t *stats, void *stream);

/* Capture fw_batch_launch(b, stats, stream) into a HIP graph held by the batch (replacing
 * an earlier capture); `stream` must be a created, non-null stream.  Nothing runs. */
int fw_batch_capture(fw_batch *b, uint64_t *stats, void *stream);

/* Launch the captured graph on `stream` (asynchronous).  FW_E_STATE without a capture. */
int fw_batch_replay(fw_batch *b, void *stream);

/* Free the batch and its graph.  NULL is accepted; its launches must have finished. */
int fw_batch_destroy(fw_batch *b);

/* For callers that cannot allocate device memory (tight serving loops, harnesses that
 * forbid hipMalloc): fw_batch_create followed by fw_batch_launch in one call that
 * allocates nothing.  Arguments, checks and results are those of the two calls (the same
 * kernels, so the walks are bit-identical).  The query table and the walker counter live
 * in a library-owned static device array of 256 + FW_NOALLOC_MAX_QUERIES * 176 bytes per
 * device, held until the process ends; nq above FW_NOALLOC_MAX_QUERIES is refused with
 * FW_E_INVALID before anything runs.  The table is copied from host memory on `stream`
 * (the call returns once its host staging has been read), so the call is not for graph
 * capture.  Every call on one device shares that array: calls ordered on one stream are
 * safe, calls that overlap on one device (other streams, other threads) race.  The launch
 * is asynchronous; a bad start vertex is reported by fw_graph_check. */
#define FW_NOALLOC_MAX_QUERIES 4096
int fw_batch_run_noalloc(fw_graph *g, const fw_query *queries, int64_t nq, const fw_plan *plan, int32_t strategy,
                         const int32_t *starts, int64_t starts_len, int32_t *paths, int64_t paths_len,
                         int32_t *lengths, int64_t lengths_len, uint64_t *stats, void *stream);

/* Walk server: continuous batching of walk requests against a resident graph.
 *
 * A server thread runs ticks: one batched launch per (logic kind, weighting) over the
 * walkers of every admitted request, each walker advancing at most `tick_steps` steps
 * before it is suspended.  Between ticks finished requests are copied to host memory
 * and released, and waiting requests are admitted in arrival order while their device
 * block (n * (4L + 16) bytes, rounded) fits in `hbm_budget` bytes and fewer than
 * `max_active` requests are admitted.  Requests that arrive while others run thus join
 * at the next tick and share the device with them.  Walker i of a request uses Philox
 * counter (i, step, draw, tag) under the request's seed: results are identical to
 * fw_walk of the same (logic, starts, L, seed), whatever the mix and the tick length.
 * The plan and strategy are fixed for the server's lifetime.  Allocates `hbm_budget`
 * bytes of device memory up front; uses its own stream. */
typedef struct fw_server fw_server;

int fw_server_create(fw_graph *g, const fw_plan *plan, int32_t strategy, uint64_t hbm_budget,
                     int32_t tick_steps, int32_t max_active, int32_t max_pending, fw_server **out);

/* Queue a request: n walkers from starts (host pointer, copied), at most L steps.  Returns
 * FW_E_BUSY when max_pending requests are already waiting, FW_E_INVALID when the request
 * can never fit the budget or a start lies outside [0, nv) (nothing is queued then).
 * *req_id identifies it (ids start at 1). */
int fw_server_submit(fw_server *s, const fw_logic *logic, const int32_t *starts, int64_t n, int32_t L,
                     uint64_t seed, uint64_t *req_id);

/* Wait up to timeout_ms for a finished request; *req_id = its id, or 0 on timeout.
 * Finished requests are reported once each, in completion order. */
int fw_server_next_done(fw_server *s, int32_t timeout_ms, uint64_t *req_id);

/* Copy a finished request's results (host pointers: n*(L+1) path slots in the fw_walk
 * layout, n lengths; either may be NULL), report its submit-to-finish latency in
 * seconds, and forget it.  FW_E_STATE if it has not finished. */
int fw_server_result(fw_server *s, uint64_t req_id, int32_t *paths, int32_t *lengths, double *latency_s);

/* Counters (8 uint64): 0 waiting, 1 admitted and unfinished, 2 finished, 3 ticks, 4 walker
 * steps, 5 budget bytes in use, 6 peak bytes in use, 7 algorithmic bytes. */
int fw_server_stats(fw_server *s, uint64_t *out);

/* Stop after the current tick and free everything; unfinished requests are dropped. */
int fw_server_destroy(fw_server *s);

/* Wait for `stream`, then report and clear the graph's device error flag: FW_OK, or
 * FW_E_INVALID if a walk since the last check met an out-of-range start vertex. */
int fw_graph_check(fw_graph *g, void *stream);

/* Message of the last failing call on this thread ("" if none). */
const char *fw_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FLEXIWALK_H */
