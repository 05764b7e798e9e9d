/*
 * mlmq.h -- C ABI of the MI355X (gfx950) Multi-Level-Multi-Queue SSSP library.
 *
 * Problem (Section 2.1): a directed graph G(V, E, W) with non-negative integer
 * edge weights and a source s; the result is L(s), the shortest path length
 * from s to every vertex. Here distances are uint32 and MLMQ_UNREACHABLE
 * (0xFFFFFFFF) marks vertices with no path from s; the largest finite distance
 * is 2^32 - 2. The result is unique, so every queue configuration, batch and
 * serving mix returns the same vector.
 *
 * Method (Sections 3-4): a persistent GPU kernel relaxes edges while its work
 * items sit in queues at three levels -- per-lane registers (L0), per-workgroup
 * LDS (L1: FIFO vector with periodic flush, near-far, or filter), and HBM (L2:
 * block FIFO or bucket queue) -- moved between levels by unified Read/Write
 * primitives, with delayed-count global termination detection.
 *
 * Conventions for every call:
 *   - Returns an int status (MLMQ_OK or a negative MLMQ_ERR_*); never throws.
 *     On failure mlmq_last_error() gives a message for the calling thread.
 *   - Out-parameters are written only on MLMQ_OK (distance buffers may have
 *     been partly written on failure).
 *   - All pointers are plain host or device addresses; sizes are element counts.
 *   - Calls may come from several host threads at once, on different streams
 *     (graphs are immutable after create; the library's queue memory pool and
 *     caches are locked). Solves return after their work on the stream is
 *     done: the call's status (capacity retry, the exact overflow test, the
 *     watchdog) is decided on the host from the device's status word, so
 *     there is no asynchronous variant of mlmq_sssp; the server
 *     (submit / poll / wait) is the asynchronous form.
 */
#ifndef MLMQ_H_
#define MLMQ_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MLMQ_OK 0
#define MLMQ_ERR_INVALID_ARG (-1)
#define MLMQ_ERR_OUT_OF_MEMORY (-2)
#define MLMQ_ERR_DISTANCE_OVERFLOW (-3)
#define MLMQ_ERR_QUEUE_CAPACITY (-4)
#define MLMQ_ERR_TIMEOUT (-5)
#define MLMQ_ERR_DEVICE (-6)
#define MLMQ_ERR_CANCELED (-7)
#define MLMQ_ERR_BUSY (-8)

#define MLMQ_UNREACHABLE 0xFFFFFFFFu

/*
 * mlmq_graph_create flags. There is no flag to borrow the caller's arrays in
 * place: the library stores each edge as one 8-byte word (column | weight <<
 * 32), so one coalesced load brings a lane both the neighbour and the weight,
 * and a caller's separate col[] / w[] arrays cannot serve as that layout.
 * Device arrays are therefore always copied (and packed) on the device.
 */
#define MLMQ_MEM_HOST 0u   /* CSR arrays are host memory; they are copied to the device */
#define MLMQ_MEM_DEVICE 1u /* CSR arrays are device memory; they are copied on the device */
/*
 * Large power-law graphs (at least 2^22 vertices, largest degree at least 16
 * times the mean) also get a second device copy whose vertex ids are
 * renumbered by decreasing degree, so that the labels of the high-degree
 * vertices, which most edges point to, share cache lines (on smaller graphs,
 * whose labels stay in cache anyway, it measured slower). Plain solves
 * (mlmq_sssp, mlmq_bfs, mlmq_autotune) run on that copy and gather the result
 * back into the caller's vertex order before they return; batches, servers,
 * mlmq_check, mlmq_latency_probe and mlmq_sssp_noalloc use the graph as given.
 * The copy costs the graph's memory once more plus 4 bytes per vertex.
 * MLMQ_GRAPH_KEEP_ORDER leaves it out; MLMQ_GRAPH_DEGREE_ORDER makes it for
 * any graph with edges. Setting both is an error.
 */
#define MLMQ_GRAPH_KEEP_ORDER 2u
#define MLMQ_GRAPH_DEGREE_ORDER 4u

/* L1 (per-workgroup LDS) queue types, Section 3.4 and Table 1 */
#define MLMQ_L1_NONE 0    /* no L1: L0 spills straight to L2 */
#define MLMQ_L1_VEC 1     /* L1V: FIFO vector, flushed to L2 after every l1_flush_wb writes */
#define MLMQ_L1_NEARFAR 2 /* L1NF: near/far vectors split at NF, NF = min(far) + delta1 */
#define MLMQ_L1_FILTER 3  /* L1FQ: keeps d <= F, the rest goes to L2; F = min(L2 batch) + delta1 */
#define MLMQ_L1_SLF 4     /* L1SLF: deque; an item shorter than the head goes in front, others at the
                             back (Small-Label-First); overflow goes to L2 */

/* Relaxation (Section 4.1's relax step): label pre-check before atomicMin, or atomicMin alone */
#define MLMQ_RELAX_PRECHECK 0
#define MLMQ_RELAX_ATOMIC 1

/* L2 (HBM) queue types, Section 4.2 and Table 1 */
#define MLMQ_L2_FIFO 0   /* L2V: block-based lock-free FIFO ring */
#define MLMQ_L2_BUCKET 1 /* L2DQ: bmax FIFO rings as buckets of width delta2 */
#define MLMQ_L2_PQ 2     /* L2PQ (pnum = 1): a heap of sorted 64-element batches with a lock per node;
                            L2MPQ (pnum > 1): pnum such heaps, each wave reading its own and writing
                            to all of them in turn */

/* Counters a solve reports (summed over all waves). */
typedef struct mlmq_stats {
  uint32_t struct_size;
  uint32_t status;         /* device status word of the last solve */
  double kernel_ms;        /* device time of init + persistent kernel (HIP events) */
  double worker_ms;        /* device time of the persistent kernel alone */
  uint64_t expansions;     /* work items that passed the stale check */
  uint64_t stale;          /* work items dropped as stale */
  uint64_t edges;          /* edges scanned */
  uint64_t pushes;         /* successful relaxations (improved distances) */
  uint64_t l1_writes;      /* L1 Write calls */
  uint64_t l1_reads;       /* L1 Read calls that returned work */
  uint64_t l2_writes;      /* L2 blocks written */
  uint64_t l2_reads;       /* L2 blocks read */
  uint64_t hub_chunks;     /* grid-cooperative edge chunks processed */
  uint64_t flushes;        /* L1V periodic flushes */
  uint32_t grid_wgs;       /* workgroups launched */
  uint32_t retries;        /* capacity retries taken */
  uint64_t donations;      /* L1 backlogs handed to L2 for idle waves */
  uint64_t atomics;        /* atomicMin issued (candidates that passed the label pre-check) */
  double wave_ms;          /* summed over waves: time spent on the query */
  double idle_ms;          /* summed over waves: time with no work at any level */
} mlmq_stats;

/*
 * Queue configuration (the search space of Section 3.5; every knob has a
 * default). Zero-initialise, set struct_size = sizeof(mlmq_config), call
 * mlmq_config_default, then change fields. Read only during a call.
 */
typedef struct mlmq_config {
  uint32_t struct_size;
  /* L0 lives in VGPRs, one element per lane per row, so its capacity is set in
     rows of 64 elements rather than in elements */
  uint8_t l0_rows;   /* L0 capacity in 64-element rows per wave, 0..4 (0 = L0 off) */
  uint8_t l1_type;   /* MLMQ_L1_* */
  uint8_t l2_type;   /* MLMQ_L2_* */
  uint8_t relax_mode; /* MLMQ_RELAX_PRECHECK: read dist[v] first, atomicMin only if it may improve;
                         MLMQ_RELAX_ATOMIC: atomicMin on every candidate (one memory round trip less
                         on the critical path; for low-degree, latency-bound graphs) */
  uint32_t l1_cap;      /* L1 capacity per workgroup in elements (power of two, 64..8192) */
  uint32_t l1_flush_wb; /* L1V: flush all of L1 to L2 after every wb L1 writes (0 = never) */
  uint32_t delta1;      /* L1NF / L1FQ threshold step (distance units, >= 1) */
  uint32_t delta2_log2; /* L2 bucket width = 2^delta2_log2 (a power of two: the bucket of a distance is
                           a shift on the hot path, not a division) */
  uint32_t bmax;        /* L2 bucket count (1..64) */
  uint32_t bnum;        /* buckets scanned per L2 read (1..bmax) */
  uint32_t th_v;        /* degree above which a whole wave expands one vertex */
  uint32_t th_hub;      /* degree above which edges are split into grid-wide chunks (0 = off) */
  uint32_t hub_chunk;   /* edges per grid-wide chunk (multiple of 64) */
  /* (the L2 block size is not a knob: a block is 64 elements, one per lane of
     the wave that writes or reads it) */
  uint32_t wg_size;     /* threads per workgroup: 64 (one wave; L1 is private to it) */
  uint32_t grid_wgs;    /* persistent workgroups (0 = as many as fit on the device) */
  uint64_t l2_capacity; /* L2 elements per query (0 = automatic); grows on overflow */
  void* stream;         /* hipStream_t to run on (NULL = null stream) */
  uint32_t timeout_ms;  /* device-side watchdog per solve (0 = 60000) */
  uint32_t max_retries; /* capacity-overflow retries with a doubled L2 (default 3) */
  mlmq_stats* stats_out; /* nullable: receives counters of the solve */
  uint32_t donate_min;  /* spill threshold for idle waves: a wave whose L1 main (near) ring holds at
                           least this many items hands the older half to L2 while other waves of the
                           query find no work (0 = automatic: 64 on graphs of >= 2^21 vertices, else
                           32; breadth-first runs 32); else 16..65536 */
  uint32_t pnum;        /* MLMQ_L2_PQ: number of priority queues, 1..64 (1 = L2PQ, more = L2MPQ) */
} mlmq_config;

typedef struct mlmq_graph mlmq_graph;   /* opaque; immutable after create */
typedef struct mlmq_server mlmq_server; /* opaque */

/* Graph features of Table 2 (Section 3.5), computed in one O(n+m) pass. */
typedef struct mlmq_features {
  double n, nnz, avg_deg, max_deg, std_deg, avg_w, std_w, max_w;
} mlmq_features;

/* Fills cfg with defaults (cfg->struct_size must be set). */
int mlmq_config_default(mlmq_config* cfg);

/*
 * Builds a device-resident graph from CSR (Section 2.1; the graph stays in HBM
 * across solves). n >= 1 vertices, m >= 0 directed edges, m < 2^31.
 * row_offsets[n+1] (row_offsets[0] = 0, non-decreasing, row_offsets[n] = m),
 * col[m] in [0, n), w[m] any uint32 (0, self-loops and parallel edges allowed).
 * flags: MLMQ_MEM_HOST or MLMQ_MEM_DEVICE tells where the arrays live; they
 * are copied, so the caller keeps ownership; MLMQ_GRAPH_KEEP_ORDER or
 * MLMQ_GRAPH_DEGREE_ORDER may be or-ed in (the degree-ordered copy, see above). Validation is O(n+m); errors give
 * MLMQ_ERR_INVALID_ARG. Needs a HIP device (else MLMQ_ERR_DEVICE).
 */
int mlmq_graph_create(int32_t n, int64_t m, const int32_t* row_offsets, const int32_t* col,
                      const uint32_t* w, uint32_t flags, mlmq_graph** out);
void mlmq_graph_destroy(mlmq_graph* g);
int mlmq_graph_info(const mlmq_graph* g, int32_t* n, int64_t* m, mlmq_features* f);

/*
 * The config a solve on g uses when cfg == NULL: the autotuned one if
 * mlmq_autotune ran, else the learned selector's top template for g's Table 2
 * features (mlmq_select), else (no model built in) defaults adjusted by the
 * features. out->struct_size must be set; stream and stats_out are left NULL.
 */
int mlmq_graph_config(const mlmq_graph* g, mlmq_config* out);

/*
 * Table 2 features of a host CSR, without a device. Same validation as
 * mlmq_graph_create.
 */
int mlmq_features_host(int32_t n, int64_t m, const int32_t* row_offsets, const int32_t* col,
                       const uint32_t* w, mlmq_features* out);

/*
 * Single-source solve (Section 2.1 / Section 4.1). dist_out: n uint32, host or
 * device memory, caller-owned; receives L(s). cfg NULL = the graph's config
 * (mlmq_graph_config: autotuned, else the selector's pick). Enqueues on cfg->stream and
 * returns after the solve finished. source >= n gives MLMQ_ERR_INVALID_ARG.
 * MLMQ_ERR_DISTANCE_OVERFLOW if a reachable vertex's distance is >= 2^32 - 1.
 * MLMQ_ERR_TIMEOUT if the device watchdog fired.
 */
int mlmq_sssp(const mlmq_graph* g, uint32_t source, uint32_t* dist_out, const mlmq_config* cfg);

/*
 * Allocation-free single-source solve, for callers that cannot allocate
 * device or pinned memory during a call (tight serving loops, harnesses that
 * forbid allocation). Same result as mlmq_sssp, but the queue memory comes
 * from one fixed device array of 128 MiB per GPU, reserved when the library
 * is loaded and held until the process ends; the call itself allocates
 * nothing (no hipMalloc, hipFree or pinned host memory). Differences from
 * mlmq_sssp:
 *   - dist_out must be device memory (n uint32), else MLMQ_ERR_INVALID_ARG;
 *   - a solve whose queue memory (the plan of mlmq_sssp's first attempt plus
 *     a few KB of control words) exceeds the 128 MiB gives
 *     MLMQ_ERR_INVALID_ARG with the size in the message; the default FIFO
 *     L2 (room for 2n elements of 8 bytes, rounded up to a power of two of
 *     64-element blocks) fits for graphs of up to 2^22 vertices;
 *   - no capacity retry: an L2 that runs out gives MLMQ_ERR_QUEUE_CAPACITY;
 *   - stats_out receives the counters but kernel_ms/worker_ms = 0.
 * Every call on a GPU uses that GPU's array, which keeps the last call's
 * contents until the next call resets it. Calls on one GPU from one process
 * therefore never overlap: the library holds a per-GPU lock for the whole
 * solve, so concurrent callers wait for each other. The call returns after
 * the solve finished on cfg->stream. Other errors as for mlmq_sssp.
 */
int mlmq_sssp_noalloc(const mlmq_graph* g, uint32_t source, uint32_t* dist_out, const mlmq_config* cfg);

/*
 * Breadth-first search levels on the same queues (Section 5.7, BFS case
 * study): levels_out[v] = fewest edges on a path from source, MLMQ_UNREACHABLE
 * where none; the weights of g are ignored. Buffers, streams and errors as for
 * mlmq_sssp. cfg NULL = the graph's config with its near-far window set to one
 * level and its bucket width to 1 (its relax mode kept: atomicMin alone on
 * low-degree graphs, with the label pre-check on power-law graphs).
 */
int mlmq_bfs(const mlmq_graph* g, uint32_t source, uint32_t* levels_out, const mlmq_config* cfg);

/*
 * Optimality check of a distance vector on the device. For positive weights a
 * vector D is the shortest-distance vector from source exactly when
 *   (1) D[source] == 0;
 *   (2) for every edge (u, v, w) with D[u] finite, D[v] is finite and
 *       D[v] <= D[u] + w (evaluated without overflow);
 *   (3) every other vertex v with D[v] finite has an edge (u, v, w) with
 *       D[u] + w == D[v]
 * (by (3) each finite D[v] is the length of a real path, by (1)-(2) no larger
 * than the shortest one; the definition of the distances of Section 2).
 * One pass reads every edge word and the labels of both ends, so its time is
 * also the cost of a single relaxation sweep of the whole graph.
 * dist: device memory, g's n uint32 (UINT32_MAX = unreachable), only read.
 * stream: hipStream_t to run on (NULL = null stream); the call blocks until
 * the check is done. *violations_out (host) receives the number of failed
 * conditions: each edge failing (2), each vertex failing (3), and 1 if (1)
 * fails; 0 means D is the exact distance vector. *edge_pass_ms_out (host,
 * may be NULL) receives the device time of the edge pass. Scratch (n bytes +
 * a counter) is allocated and freed by the call. MLMQ_ERR_INVALID_ARG for a
 * NULL argument, source >= n, or a graph with a zero-weight edge (on a cycle
 * of zero weights, (3) no longer rules out labels that are too small).
 */
int mlmq_check(const mlmq_graph* g, uint32_t source, const uint32_t* dist, void* stream, uint64_t* violations_out,
               float* edge_pass_ms_out);

/*
 * Latency probes on g's device copy, a floor for high-diameter graphs that
 * does not come from the solver itself. (1) One lane follows `hops` hops
 * from source, each hop doing the memory operations of one relaxation in
 * dependence: the row bounds of the current vertex, then one of its edge
 * words, then an agent-scope atomicMin on the neighbour's label (in a scratch
 * label array) whose returned value the next hop waits for; *hop_ns_out =
 * average time per hop. (2) Two workgroups (on different XCDs) take turns
 * incrementing one device word, each waiting to see the other's store;
 * *handoff_ns_out = one hand-off (half a round trip). stream: hipStream_t
 * (NULL = null stream); blocks until done. hops in [1, 2^24]. A solve along a
 * shortest-path tree of depth D cannot finish faster than about D hops.
 * Scratch (4n bytes) is allocated and freed by the call. MLMQ_ERR_TIMEOUT if
 * the second workgroup never answered (each wait gives up after 2 s).
 */
int mlmq_latency_probe(const mlmq_graph* g, uint32_t source, uint32_t hops, void* stream, double* hop_ns_out,
                       double* handoff_ns_out);

/*
 * Many queries in one persistent launch. Query i solves graphs[i] from
 * sources[i] into dist_outs[i] (device memory, n_i uint32 each). cfgs may be
 * NULL (per-graph autotuned/default) or hold one config per query; launch
 * shape and stream come from cfgs[0] (or defaults). per_query_status may be
 * NULL or receive each query's status. Output per query is identical to
 * mlmq_sssp alone. Returns the first non-OK query status, else MLMQ_OK.
 */
int mlmq_sssp_batch(const mlmq_graph* const* graphs, const uint32_t* sources, uint32_t* const* dist_outs,
                    int32_t nq, const mlmq_config* const* cfgs, int32_t* per_query_status);

/*
 * Input-adaptive configuration (Section 3.5). The library holds a fixed list
 * of candidate configurations ("templates"): each L1 policy over each L2 type,
 * with and without register queues, with the near-far/filter step, bucket
 * width, L1 capacity, launch size, donation threshold, L1V flush period and
 * whole-wave threshold set relative to the graph's Table 2 features or to the
 * device. A learned selector -- a random-forest regressor trained offline on
 * timings of every template over a seeded synthetic corpus of grids, RMAT and
 * uniform graphs -- predicts each template's runtime relative to the best
 * template on that graph from the Table 2 features and the template's knobs.
 * The workgroup size is not searched: a workgroup is always one wave64.
 */

/* Number of templates (ids 0 .. count-1). */
int32_t mlmq_candidate_count(void);

/*
 * Template t as a config for graph g (t = -1: the feature-driven default,
 * which cfg == NULL falls back to without a model). out->struct_size must be set; its
 * stream and stats_out are kept. Needs a device (the launch size depends on
 * its compute units). MLMQ_ERR_INVALID_ARG for t out of range.
 */
int mlmq_candidate_config(const mlmq_graph* g, int32_t t, mlmq_config* out);

/*
 * Host only (no device needed). x receives the selector's 20 model inputs for
 * template t on a graph with features f (the Table 2 features, sizes as log2,
 * spreads relative to their means, then the template's knobs); the training
 * script builds its data with this call.
 */
int mlmq_select_inputs(const mlmq_features* f, int32_t t, float* x);

/*
 * Host only. Ranks the templates for features f by the selector's predicted
 * relative performance: order[0 .. min(cap, count)) receives template ids,
 * best first (ties in list order); scores (nullable, count floats) receives
 * each template's prediction (1 = as fast as the best template).
 */
int mlmq_select_rank(const mlmq_features* f, int32_t* order, float* scores, int32_t cap);

/*
 * The selector's top template for g as a config, without timing anything
 * (the feature-driven default if no model is built in); it is what cfg ==
 * NULL uses until mlmq_autotune caches a timed choice. out->struct_size must
 * be set; stream and stats_out are kept.
 */
int mlmq_select(const mlmq_graph* g, mlmq_config* out);

/*
 * Autotuner (Section 3.5's input-adaptive configuration, measured): the
 * feature-driven default, then the templates in the selector's order, each
 * timed on three seeded sources (the highest-degree vertex and two drawn
 * among vertices with edges) until budget_ms is spent (0 = 2000); a candidate
 * may not run longer than 4x the best total so far. The fastest is cached for
 * the graph (used by cfg == NULL) and written to *out (nullable; struct_size
 * must be set; its stream, used for the timing runs, and stats_out are kept).
 */
int mlmq_autotune(mlmq_graph* g, uint32_t budget_ms, mlmq_config* out);

/*
 * Continuous-batching server over resident graphs (the serving form of the
 * Section 4.1 persistent kernel): a resident kernel picks up queries from a
 * table of max_slots (1..64) slots while others run; its idle waves sleep, the
 * library stops the whole kernel after 200 ms with no query pending or running
 * and relaunches it when work arrives. Queries are admitted in arrival order when a slot is free and their
 * state (queues + n distances) fits in mem_budget_bytes; a query larger than
 * the budget runs alone. Each graph uses cfg if given, else its own config
 * (mlmq_graph_config); graphs must outlive the server. submit never blocks
 * (MLMQ_ERR_BUSY if 2^20 queries are pending); dist_out is device memory of
 * graphs[graph_id]'s n uint32 that the caller keeps valid until the query
 * finished. Each result is identical to mlmq_sssp of the same query alone.
 * The library's streams are non-blocking; hipDeviceSynchronize waits for the
 * resident kernel, so callers use stream or event synchronisation while a
 * server is alive. destroy cancels pending queries, waits for running ones
 * and stops the kernel. cfg (nullable) replaces every graph's config (one
 * resident kernel serves all graphs; NULL = each graph's own config).
 */
int mlmq_server_create(const mlmq_graph* const* graphs, int32_t ngraphs, uint64_t mem_budget_bytes,
                       int32_t max_slots, const mlmq_config* cfg, mlmq_server** out);
int mlmq_server_submit(mlmq_server* s, int32_t graph_id, uint32_t source, uint32_t* dist_out,
                       uint64_t* ticket);
/* Non-blocking; *done_status = 1 (not finished) or the query's final status. */
int mlmq_server_poll(mlmq_server* s, uint64_t ticket, int32_t* done_status);
/* Blocks up to timeout_ms; returns the query's status or MLMQ_ERR_TIMEOUT. */
int mlmq_server_wait(mlmq_server* s, uint64_t ticket, uint32_t timeout_ms);
/* Timestamps (ns, host monotonic clock) of submission and completion. */
int mlmq_server_times(mlmq_server* s, uint64_t ticket, uint64_t* submit_ns, uint64_t* done_ns);
void mlmq_server_destroy(mlmq_server* s);

/* Message for the calling thread's last non-OK return. */
const char* mlmq_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MLMQ_H_ */
