// Internal layout shared by the host side of the library and its HIP kernels.
// Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlmq {

constexpr int kWave = 64;               // CDNA wavefront width
constexpr uint32_t kInf = 0xFFFFFFFFu;  // unreachable / "no ticket"
constexpr int kMaxBuckets = 64;         // L2 buckets: one per lane of a scanning wave
constexpr int kMaxL0Rows = 4;           // L0 register rows of 64 elements
constexpr uint32_t kStageB = 8;         // buckets after the head with a write-combining row

// Device status word of a query (ctrl->error).
enum : uint32_t {
  kStOk = 0,
  kStCapacity = 1,     // an L2 ring had no free block
  kStHubCapacity = 2,  // the grid-wide chunk table was full
  kStTimeout = 3,      // device watchdog fired
  kStCanceled = 4,     // host asked the kernel to stop
};

// Counters summed into QueryCtrl::stats (order matches mlmq_stats).
enum : int {
  kCtExpansions = 0,
  kCtStale,
  kCtEdges,
  kCtPushes,
  kCtL1Writes,
  kCtL1Reads,
  kCtL2Writes,
  kCtL2Reads,
  kCtHubChunks,
  kCtFlushes,
  kCtDonations,
  kCtAtomics,    // atomicMin issued (candidates that passed the label pre-check)
  kCtWaveTicks,  // wall-clock ticks the waves spent on the query
  kCtIdleTicks,  // of which with no work at any level
  kNumCounters
};

// One independently-updated 32-bit word per 128-byte line, so that counters
// hammered by different waves never share a cache line.
struct alignas(128) Word {
  uint32_t v;
  uint32_t pad[31];
};

// Per-query control block (device memory, reset by the init kernel).
struct QueryCtrl {
  Word done;       // L2 blocks + hub chunks fully processed (delayed count)
  Word terminate;  // 1 once the queue system is empty
  Word error;      // first kSt* error
  Word overflow;   // some candidate distance did not fit in 32 bits
  Word cur;        // absolute index of the head L2 bucket
  Word hub_tail;   // hub records allocated
  Word hub_head;   // first hub record that may still have chunks
  Word hub_units;  // hub chunks reserved (termination count)
  Word joined;     // workgroups that joined this query
  Word finished;   // workgroups that left this query (server queries: low 16 bits; the high
                   // 16 bits hold the number of waves on the query, set by the first to leave)
  Word hungry;     // waves of this query that currently find no work
  Word active;     // waves currently working on this query
  Word pq_in;      // elements written to the L2 priority queues (termination count)
  uint64_t stats[16];  // [0, kNumCounters) used
};

// L2 ring counters: tickets handed to writers (tail) and readers (head).
// For the L2 priority queues, tail holds the number of heap nodes in use.
struct RingCtr {
  Word tail;
  Word head;
};

// Everything a workgroup needs to work on one query. Device memory, one per
// query; loaded into scalar registers by the kernel.
struct QueryDesc {
  const int32_t* off;  // CSR row offsets [n+1]
  const uint64_t* adj; // CSR edges [m]: col | (weight << 32)
  uint32_t* dist;      // output distances [n]
  QueryCtrl* ctrl;
  RingCtr* rings;      // [nrings]
  uint64_t* hdr;       // [nrings << nb_log2] block headers: (seq << 32) | count;
                       // priority queues: node words, lock (low 32 bits) and state (high)
  uint64_t* data;      // [(nrings << nb_log2) * 64] elements: v | (d << 32)
  uint64_t* hub_rec;   // [2 * hub_cap] records: (v | d << 32), (beg | end << 32)
  uint32_t* hub_cur;   // [hub_cap] chunk claim cursors
  uint32_t* hub_pub;   // [hub_cap] 1 once the record is readable
  uint32_t n;
  uint32_t source;
  uint32_t nb_log2;    // blocks per ring = 1 << nb_log2
  uint32_t nrings;     // 1 (FIFO), bmax (bucket) or pnum (priority queues)
  uint32_t hub_cap;
  uint32_t l0_cap;     // L0 elements per wave (rows * 64), 0 = off
  uint32_t l1_type;
  uint32_t l2_type;
  uint32_t l1_cap;     // power of two
  uint32_t l1_wb;
  uint32_t delta1;
  uint32_t d2_log2;
  uint32_t bnum;
  uint32_t th_v;
  uint32_t th_hub;     // 0 = hub tier off
  uint32_t hub_chunk;
  uint32_t want_wgs;   // workgroups this query should get
  uint32_t relax_mode; // MLMQ_RELAX_*
  uint32_t unit_w;     // 1: every edge weighs 1 (breadth-first levels)
  uint32_t donate_min; // near-ring size from which a wave hands half of it to idle waves
};

// Batch-wide control (device memory).
struct BatchCtrl {
  Word cursor;  // first query that may still accept workgroups
  Word cancel;  // host sets 1 to stop the launch
};

struct LaunchArgs {
  const QueryDesc* queries;
  BatchCtrl* batch;
  int32_t nq;
  uint32_t l1_cap;     // LDS ring capacity this launch was sized for
  uint32_t l1_two;     // 1 if a second (far) ring is allocated
  uint32_t stage;      // 1 if the bucket-queue write-combining area is allocated
  uint32_t waves;      // waves per workgroup (always 1)
  uint32_t pq;         // 1: the kernel variant with the L2 priority-queue code
  uint64_t timeout_ticks;   // device watchdog (wall-clock ticks)
  uint64_t cap_wait_ticks;  // longest wait for a free L2 slot before overflow
  uint32_t* beats;          // [grid] last program point of each wave (nullable)
};

// Control words of a resident server kernel (device memory).
struct ServerCtrl {
  Word stop;       // 1: idle waves leave the kernel
  Word cancel;     // 1: every query stops (status canceled)
  Word last_busy;  // low 32 bits of the wall clock when a wave last joined or left a query
};

struct ServerArgs {
  const QueryDesc* slots;  // [nslots] descriptors, rewritten on admission
  uint64_t* join;          // [nslots] slot words (see the server kernel)
  uint64_t* done_host;     // [nslots] host-coherent: (status << 32) | generation
  ServerCtrl* ctl;
  int32_t nslots;          // <= 64
  uint32_t l1_cap;         // LDS ring capacity the launch was sized for
  uint32_t l1_two;         // 1 if a second (far) ring is allocated
  uint32_t stage;          // 1 if the bucket-queue write-combining area is allocated
  uint32_t pq;             // 1: the kernel variant with the L2 priority-queue code
  uint64_t timeout_ticks;  // per-query device watchdog from the moment a wave joins
  uint64_t cap_wait_ticks;
  uint64_t idle_exit_ticks;  // a wave with no work for this long leaves the kernel
};

// Program points a wave reports in its heartbeat word (point << 24 | iteration).
enum : uint32_t {
  kPtPick = 1,
  kPtLoop = 2,
  kPtHub = 3,
  kPtL2Read = 4,
  kPtIdle = 5,
  kPtProcess = 6,
  kPtL2Wait = 7,
  kPtDone = 8,
};

// Compact per-query outcome gathered after a batch launch.
struct QueryResult {
  uint32_t error;
  uint32_t overflow;
  uint64_t stats[kNumCounters];
};

// Bytes of dynamic LDS a workgroup needs.
size_t worker_lds_bytes(uint32_t waves, uint32_t l1_cap, bool two_rings, bool stage);

// Kernel launchers (defined in mlmq_kernels.hip).
hipError_t launch_init(const QueryDesc* d_queries, BatchCtrl* d_batch, int nq, uint32_t max_words, hipStream_t s);
hipError_t launch_worker(const LaunchArgs& a, uint32_t grid, uint32_t wg_size, size_t lds, hipStream_t s);
hipError_t launch_overflow_check(const QueryDesc* d_query, uint32_t* d_flag, hipStream_t s);
// out[v] = lab[ord_of[v]] for v < n (labels of a degree-ordered solve, back in the caller's order)
hipError_t launch_unorder(const uint32_t* d_lab, const uint32_t* d_ord_of, uint32_t n, uint32_t* d_out, hipStream_t s);
hipError_t launch_gather(const QueryDesc* d_queries, int nq, QueryResult* d_out, hipStream_t s);
hipError_t worker_occupancy(uint32_t wg_size, size_t lds, bool pq, int* wgs_per_cu);
hipError_t launch_server_worker(const ServerArgs& a, uint32_t grid, size_t lds, hipStream_t s);
// Resets the query's memory, stores its descriptor in *d_slot, then stores
// word into *d_join (two kernels in stream order).
hipError_t launch_server_admit(const QueryDesc& q, QueryDesc* d_slot, uint64_t* d_join, uint64_t word,
                               uint32_t max_words, hipStream_t s);
hipError_t launch_server_signal(uint32_t* d_word, uint32_t v, hipStream_t s);
// Optimality check of a distance vector (edge pass timed between ev0 and ev1,
// then the vertex pass); tight (n bytes) and *bad must be zero on entry.
hipError_t launch_check(const int32_t* off, const uint64_t* adj, const uint32_t* dist, uint32_t n, uint32_t m,
                        uint32_t source, uint8_t* tight, unsigned long long* bad, hipEvent_t ev0, hipEvent_t ev1,
                        hipStream_t s);
hipError_t server_occupancy(size_t lds, bool pq, int* wgs_per_cu);
// Latency probes: a dependent-hop chain of `hops` relaxations from v0 over
// labels lab[n] (out[0] = ticks), then `rounds` hand-off round trips between
// two workgroups on *word (out[2] = ticks, out[3] = 1 if it gave up); word
// and out must be zero on entry.
hipError_t launch_latency_probes(const int32_t* off, const uint64_t* adj, uint32_t* lab, uint32_t n, uint32_t v0,
                                 uint32_t hops, uint32_t* word, uint32_t rounds, uint64_t limit_ticks, uint64_t* out,
                                 hipStream_t s);

// Bytes of the fixed device array behind the allocation-free solve.
constexpr size_t kNoAllocScratchBytes = 128ull << 20;
// Device address of that array on `device`, which must be the current device;
// looked up once per device and cached.
hipError_t noalloc_scratch(int device, void** out);

}  // namespace mlmq
