// Multi-Level-Multi-Queue SSSP kernels for CDNA4 (gfx950).
//
// One persistent kernel relaxes edges while work items (vertex, distance)
// live in three levels of queues (Section 3.1):
//   L0  per wave, in VGPRs: a ring of up to 4 rows x 64 lanes, FIFO;
//   L1  per workgroup, in LDS: FIFO vector with periodic flush, near-far pair
//       or filter (Section 3.4). A workgroup is one wave64, so L1 is private
//       to its wave like the paper's per-warp L1 and needs no lock;
//   L2  per query, in HBM: block-based FIFO ring(s) with ticket counters
//       (Section 4.2), one ring for L2V or bmax rings used as Delta buckets
//       for L2DQ; or pnum batched heaps with per-node locks (L2PQ, and the
//       multi-queue L2MPQ for pnum > 1), compiled into a second kernel
//       variant only.
// The worker only talks to the unified Read/Write cascade (Section 3.2-3.3):
// Read takes from L0, else L1, else the global levels; Write appends to L0,
// whose overflow moves everything to L1, whose overflow goes to L2.
// Termination uses delayed counting (Section 4.1): every L2 block (and every
// grid-wide hub chunk) is reserved when it is written; a wave adds what it
// took from the global levels to the done count only when it holds nothing
// (L0 and L1 empty, the global read came back empty); the query is finished
// when done equals the number reserved.
//
// Memory ordering across the 8 XCDs: queue payloads and headers are written
// and read with agent-scope relaxed atomics, which gfx950 issues with the sc1
// bit, and publication is ordered by waiting for the payload stores
// (s_waitcnt vmcnt(0)) before the header store. Distances only ever decrease,
// so plain (possibly stale) loads of dist[] are safe filters; the
// authoritative update is the atomicMin.
//
// Every wait is bounded by the device watchdog deadline and the host's cancel
// flag, and every cross-lane operation runs with the whole wave active.

#include "mlmq_internal.h"

#include <mutex>

#include "../../include/mlmq.h"

namespace mlmq {
namespace {

// ------------------------------------------------------------ wave helpers

__device__ __forceinline__ uint32_t lane() { return __lane_id(); }
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ uint32_t popc(uint64_t m) { return (uint32_t)__popcll(m); }
__device__ __forceinline__ uint32_t first_lane(uint64_t m) { return (uint32_t)__ffsll((long long)m) - 1; }
__device__ __forceinline__ uint32_t rank_of(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint32_t lane_val(uint32_t x, uint32_t l) { return __builtin_amdgcn_readlane(x, l); }
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
  return ((uint64_t)uni((uint32_t)(x >> 32)) << 32) | uni((uint32_t)x);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t x) {
#pragma unroll
  for (int o = 32; o; o >>= 1) x += __shfl_xor(x, o);
  return x;
}
__device__ __forceinline__ uint32_t wave_min(uint32_t x) {
#pragma unroll
  for (int o = 32; o; o >>= 1) x = min(x, (uint32_t)__shfl_xor(x, o));
  return x;
}
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o);
    if (lane() >= (uint32_t)o) x += y;
  }
  return x;
}

// Coherent (agent-scope) accesses: sc1 loads/stores, device-wide atomics.
__device__ __forceinline__ uint32_t ld32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t add32(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool cas32(uint32_t* p, uint32_t expect, uint32_t v) {
  return __hip_atomic_compare_exchange_strong(p, &expect, v, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
}
// Plain cached load of a distance label (may be stale, i.e. too large).
__device__ __forceinline__ uint32_t ld_label(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
// Wait until every vector memory operation of this wave has completed.
__device__ __forceinline__ void vm_drain() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
__device__ __forceinline__ void compiler_fence() { asm volatile("" ::: "memory"); }

__device__ __forceinline__ uint32_t elem_v(uint64_t e) { return (uint32_t)e; }
__device__ __forceinline__ uint32_t elem_d(uint64_t e) { return (uint32_t)(e >> 32); }
__device__ __forceinline__ uint64_t make_elem(uint32_t v, uint32_t d) { return (uint64_t)v | ((uint64_t)d << 32); }
__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b) { return a > kInf - b ? kInf : a + b; }

// Sleep for roughly 64 * 2^level cycles (level 0..6); level is wave-uniform,
// so exactly one s_sleep runs.
__device__ __forceinline__ void backoff(uint32_t level) {
  switch (uni(level)) {
    case 0: __builtin_amdgcn_s_sleep(1); break;
    case 1: __builtin_amdgcn_s_sleep(2); break;
    case 2: __builtin_amdgcn_s_sleep(4); break;
    case 3: __builtin_amdgcn_s_sleep(8); break;
    case 4: __builtin_amdgcn_s_sleep(16); break;
    case 5: __builtin_amdgcn_s_sleep(32); break;
    default: __builtin_amdgcn_s_sleep(64); break;
  }
}

// ------------------------------------------------------------ wave state

struct Ctx {
  QueryDesc q;
  uint64_t* stg;  // 64-entry staging row (LDS)
  uint64_t* l1;   // L1 main (or near) ring (LDS)
  uint64_t* far;  // L1 far ring (LDS, near-far only)
  uint64_t* stage;  // bucket write-combining rows, kStageB x 64 (LDS, bucket L2 only)
  uint32_t sb;      // lane s < kStageB: absolute bucket held in row s (kInf = none)
  uint32_t sn;      // lane s < kStageB: elements in row s
  uint32_t l1mask;
  uint32_t qh, qt, fh, ft;   // L1 ring counters (monotonic)
  uint32_t thresh;           // NF (near-far) or F (filter)
  uint32_t wcount;           // L1 writes since the last periodic flush
  uint32_t done_acc;         // blocks / hub chunks taken, not yet added to done
  uint32_t pend;             // lane r: claimed but unpublished ticket of ring r; with one ring,
                             // lane 1: claims still allowed without reading its counters (kInf = none)
  const uint32_t* cancel;    // host-set flag: stop now
  uint64_t deadline;         // device watchdog (wall-clock ticks)
  uint64_t cap_wait;         // longest wait for a free L2 slot
  uint64_t r0, r1, r2, r3;   // L0 rows (per lane)
  uint32_t l0h, l0n;         // L0 head position and count
  uint32_t* beat;            // this wave's heartbeat word (nullable)
  uint32_t it;               // loop iterations (heartbeat)
  bool pq;                   // the query's L2 is the priority queue(s) (PQ kernel variant only)
  uint32_t rq, wq;           // priority queues: this wave's reading queue, next queue written
  bool stop;                 // leave the query (terminated or failed)
  bool ovf;                  // a candidate distance overflowed
  bool hungry;               // this wave is counted in ctrl->hungry
  uint32_t idle;             // consecutive loop iterations without work
  uint64_t ct64_wave, ct64_idle;  // ticks on the query / idle (set when it ends)
  uint32_t ct[kNumCounters]; // per-wave counters
};

__device__ __forceinline__ void fail(Ctx& c, uint32_t code) {
  if (lane() == 0) {
    cas32(&c.q.ctrl->error.v, kStOk, code);
    st32(&c.q.ctrl->terminate.v, 1u);
  }
  c.stop = true;
}

// Heartbeat: written through to memory so the host can read it while the
// kernel runs (a diagnostic for the host watchdog).
__device__ __forceinline__ void beat(uint32_t* b, uint32_t point, uint32_t it) {
  if (b && lane() == 0)
    __hip_atomic_store(b, (point << 24) | (it & 0xFFFFFFu), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
// Program points inside the worker loop report on one iteration in 64 only:
// a wave that is stuck still reports within 64 turns of its loop, and the
// store stays off the per-iteration path.
__device__ __forceinline__ void beat_loop(uint32_t* b, uint32_t point, uint32_t it) {
  if ((it & 63u) == 0) beat(b, point, it);
}

__device__ __forceinline__ bool past_deadline(const Ctx& c) { return (uint64_t)wall_clock64() > c.deadline; }
__device__ __forceinline__ bool canceled(const Ctx& c) { return uni(ld32(c.cancel)) != 0; }

// Watchdog and cancel test; true if the wave must leave the query.
__device__ __forceinline__ bool must_stop(Ctx& c) {
  if (uni(ld32(&c.q.ctrl->terminate.v))) return true;
  if (past_deadline(c)) {
    fail(c, kStTimeout);
    return true;
  }
  if (canceled(c)) {
    fail(c, kStCanceled);
    return true;
  }
  return false;
}

// ------------------------------------------------------------ L0 (VGPR ring)

// Rows are picked with masks rather than an index, so no row is ever
// addressed through memory and all four stay in VGPRs.
__device__ __forceinline__ uint64_t row_mask(uint32_t row, uint32_t i) { return 0ull - (uint64_t)(row == i); }
__device__ __forceinline__ uint64_t l0_get(const Ctx& c, uint32_t row) {
  return (c.r0 & row_mask(row, 0)) | (c.r1 & row_mask(row, 1)) | (c.r2 & row_mask(row, 2)) |
         (c.r3 & row_mask(row, 3));
}
__device__ __forceinline__ void l0_set(Ctx& c, uint32_t row, uint64_t x, bool p) {
  const uint64_t keep = p ? 0ull : ~0ull;
  const uint64_t m0 = row_mask(row, 0) & ~keep, m1 = row_mask(row, 1) & ~keep;
  const uint64_t m2 = row_mask(row, 2) & ~keep, m3 = row_mask(row, 3) & ~keep;
  c.r0 = (c.r0 & ~m0) | (x & m0);
  c.r1 = (c.r1 & ~m1) | (x & m1);
  c.r2 = (c.r2 & ~m2) | (x & m2);
  c.r3 = (c.r3 & ~m3) | (x & m3);
}
// L0 Read: up to 64 elements from the head; lane j gets the one element of the
// window whose ring position is congruent to j (mod 64), so no lane movement.
__device__ __forceinline__ void l0_read(Ctx& c, uint64_t& e, bool& ok) {
  const uint32_t cap = c.q.l0_cap;
  const uint32_t k = min(c.l0n, 64u);
  const uint32_t off = (lane() - c.l0h) & 63u;
  ok = off < k;
  uint32_t pos = c.l0h + off;
  if (pos >= cap) pos -= cap;
  e = l0_get(c, pos >> 6);
  c.l0h += k;
  if (c.l0h >= cap) c.l0h -= cap;
  c.l0n -= k;
}
// Compact the lanes with ok into the staging row, in lane order.
__device__ __forceinline__ void stage(Ctx& c, uint64_t e, bool ok) {
  const uint64_t m = ballot(ok);
  if (ok) c.stg[rank_of(m)] = e;
  compiler_fence();
}
// L0 Write: append the k staged elements at the tail (caller ensures room).
__device__ __forceinline__ void l0_append(Ctx& c, uint32_t k) {
  const uint32_t cap = c.q.l0_cap;
  uint32_t base = c.l0h + c.l0n;
  if (base >= cap) base -= cap;
  const uint32_t off = (lane() - base) & 63u;
  const bool p = off < k;
  const uint64_t x = p ? c.stg[off] : 0;
  uint32_t pos = base + off;
  if (pos >= cap) pos -= cap;
  l0_set(c, pos >> 6, x, p);
  c.l0n += k;
  compiler_fence();
}

// ------------------------------------------------------------ L2 (HBM rings)

// Write one block of up to 64 elements to ring `ring` (Section 4.2, L2 FIFO:
// one atomicAdd per block). The ticket counter doubles as the termination
// reservation. Slot states: 2*lap = free for lap, 2*lap+1 = full for lap.
__device__ __forceinline__ bool l2_put_block(Ctx& c, uint32_t ring, uint64_t e, bool ok, uint64_t m) {
  const uint32_t k = popc(m);
  uint32_t t = 0;
  if (lane() == 0) t = add32(&c.q.rings[ring].tail.v, 1u);
  t = lane_val(t, 0);
  const uint32_t nb = c.q.nb_log2;
  const uint32_t slot = t & ((1u << nb) - 1u);
  const uint32_t lap = t >> nb;
  const uint64_t bidx = ((uint64_t)ring << nb) + slot;
  uint64_t* h = c.q.hdr + bidx;
  // The slot is reusable once the previous lap's reader released it; a ring
  // that stays full for longer than the capacity wait is an overflow.
  uint64_t t_wait = 0;
  for (uint32_t spins = 0;; ++spins) {
    const uint32_t seq = uni((uint32_t)(ld64(h) >> 32));
    if (seq == 2u * lap) break;
    if ((spins & 63u) == 0) {
      beat(c.beat, kPtL2Wait, spins);
      const uint64_t now = (uint64_t)wall_clock64();
      if (spins == 0) t_wait = now;
      if (now > c.deadline) {
        fail(c, kStTimeout);
        return false;
      }
      if (now - t_wait > c.cap_wait) {
        fail(c, kStCapacity);
        return false;
      }
    }
    __builtin_amdgcn_s_sleep(2);
  }
  uint64_t* dst = c.q.data + (bidx << 6);
  if (ok) st64(dst + rank_of(m), e);
  vm_drain();
  if (lane() == 0) st64(h, ((uint64_t)(2u * lap + 1u) << 32) | k);
  c.ct[kCtL2Writes] += 1;
  return true;
}

// ------------------------------------------------------------ L2 priority queues (L2PQ / L2MPQ)
//
// Section 4.2's warp-level priority queue in the spirit of a batched heap:
// a complete binary tree of nodes, each holding a sorted batch of 64
// elements, every node with its own lock; a node's elements are no larger
// than its children's when no operation is passing through. The batch of a
// node is read and written by the whole wave (lane i holds element i) and
// batches are combined by bitonic merges across lanes. Node 0 of a queue is
// a partial buffer of fewer than 64 elements; it, the node count and node 1
// are guarded by node 1's lock.
//   Write: merge the new elements into the partial buffer; once it reaches 64,
//     its 64 smallest go down the tree: the node count grows by one (the
//     new last node is marked as the target), and the batch is merged into
//     each node on the path from the root to the target, each keeping its
//     smaller half, locks taken parent before child (hand over hand).
//   Read: the root's batch merged with the partial buffer gives the 64
//     smallest elements; the last node's batch (waiting, with the root held,
//     until an insertion on its way there has arrived) replaces the root and
//     sinks: at each node the two children are merged, the child with the
//     larger maximum keeps the larger half, and the node keeps the smallest
//     64 of itself and the smaller half while the other child takes the rest
//     and the descent continues there.
// Every lock is taken in tree order (a parent before its children, the left
// child before the right), so waits cannot form a cycle; the only other wait,
// a reader holding the root for an insertion on its way to the last node,
// waits for a wave that needs no lock above that node. All waits are bounded
// by the watchdog and the cancel flag. Termination counts elements: pq_in
// grows by k before k elements are written, done by the elements read.
// L2MPQ (pnum > 1, after the multi-queue designs the paper cites): each wave
// reads from queue blockIdx mod pnum and writes to the queues in turn,
// starting at its reading queue; a wave whose reading queue is empty tries
// the others once before it counts as idle, so no element is left in a queue
// whose readers are busy elsewhere.

constexpr uint64_t kKeyInf = ~0ull;
enum : uint32_t { kNodeEmpty = 0, kNodeFull = 1, kNodeTarget = 2 };

__device__ __forceinline__ uint64_t shfl64(uint64_t x, uint32_t src) {
  const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)x, (int)src);
  const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(x >> 32), (int)src);
  return (uint64_t)lo | ((uint64_t)hi << 32);
}
__device__ __forceinline__ uint64_t shfl_xor64(uint64_t x, uint32_t m) { return shfl64(x, lane() ^ m); }
__device__ __forceinline__ uint64_t min64(uint64_t a, uint64_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint64_t max64(uint64_t a, uint64_t b) { return a < b ? b : a; }

// Ascending bitonic sort of the wave's 64 keys (lane i ends with the i-th smallest).
__device__ __forceinline__ uint64_t sort64(uint64_t x) {
#pragma unroll
  for (uint32_t k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (uint32_t j = k >> 1; j; j >>= 1) {
      const uint64_t y = shfl_xor64(x, j);
      const bool up = (lane() & k) == 0u || k == 64u;
      const bool low = (lane() & j) == 0u;
      x = (low == up) ? min64(x, y) : max64(x, y);
    }
  }
  return x;
}

// Sorts a bitonic sequence held one key per lane into ascending order.
__device__ __forceinline__ uint64_t bitonic_clean(uint64_t x) {
#pragma unroll
  for (uint32_t j = 32; j; j >>= 1) {
    const uint64_t y = shfl_xor64(x, j);
    x = (lane() & j) == 0u ? min64(x, y) : max64(x, y);
  }
  return x;
}

// Merge of two ascending batches: lo gets the 64 smallest of the 128 keys,
// hi the 64 largest, both ascending.
__device__ __forceinline__ void merge64(uint64_t a, uint64_t b, uint64_t& lo, uint64_t& hi) {
  const uint64_t br = shfl64(b, 63u - lane());
  lo = bitonic_clean(min64(a, br));
  hi = bitonic_clean(max64(a, br));
}

__device__ __forceinline__ uint64_t* pq_word(const Ctx& c, uint32_t q, uint32_t i) {
  return c.q.hdr + (((uint64_t)q << c.q.nb_log2) + i);
}
__device__ __forceinline__ uint32_t* pq_lock(const Ctx& c, uint32_t q, uint32_t i) {
  return reinterpret_cast<uint32_t*>(pq_word(c, q, i));
}
__device__ __forceinline__ uint32_t* pq_state(const Ctx& c, uint32_t q, uint32_t i) {
  return reinterpret_cast<uint32_t*>(pq_word(c, q, i)) + 1;
}
__device__ __forceinline__ uint64_t* pq_keys(const Ctx& c, uint32_t q, uint32_t i) {
  return c.q.data + ((((uint64_t)q << c.q.nb_log2) + i) << 6);
}
__device__ __forceinline__ uint64_t pq_load(const Ctx& c, uint32_t q, uint32_t i) {
  return ld64(pq_keys(c, q, i) + lane());
}
__device__ __forceinline__ void pq_store(const Ctx& c, uint32_t q, uint32_t i, uint64_t x) {
  st64(pq_keys(c, q, i) + lane(), x);
}

// Bounded wait for a node lock (false: the query failed meanwhile, or, with
// tries != 0, the lock stayed busy for that many looks). The lock word is
// read first and swapped only when it looks free, and the pause between looks
// grows, so thousands of waiting waves do not flood the root's lock with
// atomics (which would delay the holder's own release behind them).
__device__ __forceinline__ bool pq_acquire(Ctx& c, uint32_t* lk, uint32_t tries = 0) {
  for (uint32_t spins = 0;; ++spins) {
    uint32_t got = 0;
    if (lane() == 0) got = (ld32(lk) == 0u && cas32(lk, 0u, 1u)) ? 1u : 0u;
    if (lane_val(got, 0)) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      return true;
    }
    if (tries && spins + 1u >= tries) return false;
    if ((spins & 15u) == 15u && must_stop(c)) {
      c.stop = true;
      return false;
    }
    backoff(min(spins >> 1, 6u));
  }
}
// Stores of the node's data complete before its lock is free again.
__device__ __forceinline__ void pq_release(uint32_t* lk) {
  vm_drain();
  if (lane() == 0) __hip_atomic_store(lk, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Sinks the batch x just placed at node i (locked by the caller) until the
// heap order holds below it; releases every lock it took.
__device__ __forceinline__ void pq_sink(Ctx& c, uint32_t q, uint32_t i, uint64_t x) {
  const uint32_t cap = (1u << c.q.nb_log2) - 1u;
  for (;;) {
    const uint32_t l = 2u * i, r = l + 1u;
    bool hl = false, hr = false;
    if (l <= cap) {
      if (!pq_acquire(c, pq_lock(c, q, l))) return;
      hl = uni(ld32(pq_state(c, q, l))) == kNodeFull;
      if (!hl) pq_release(pq_lock(c, q, l));
    }
    if (r <= cap) {
      if (!pq_acquire(c, pq_lock(c, q, r))) return;
      hr = uni(ld32(pq_state(c, q, r))) == kNodeFull;
      if (!hr) pq_release(pq_lock(c, q, r));
    }
    if (!hl && !hr) {
      pq_release(pq_lock(c, q, i));
      return;
    }
    uint32_t keep = 0, next = 0;  // child given its final batch, child the descent continues in
    uint64_t small;
    if (hl && hr) {
      const uint64_t a = pq_load(c, q, l), b = pq_load(c, q, r);
      uint64_t lo, hi;
      merge64(a, b, lo, hi);
      const bool left_big = shfl64(a, 63) >= shfl64(b, 63);
      keep = left_big ? l : r;
      next = left_big ? r : l;
      pq_store(c, q, keep, hi);
      pq_release(pq_lock(c, q, keep));
      small = lo;
    } else {
      next = hl ? l : r;
      small = pq_load(c, q, next);
    }
    if (shfl64(x, 63) <= shfl64(small, 0)) {  // already in order
      if (hl && hr) pq_store(c, q, next, small);
      pq_release(pq_lock(c, q, next));
      pq_release(pq_lock(c, q, i));
      return;
    }
    uint64_t lo, hi;
    merge64(x, small, lo, hi);
    pq_store(c, q, i, lo);
    pq_store(c, q, next, hi);
    pq_release(pq_lock(c, q, i));
    i = next;
    x = hi;
  }
}

// Inserts a full sorted batch into queue q; the caller holds the root lock,
// which this releases (with every other lock it takes).
__device__ __forceinline__ void pq_push_full(Ctx& c, uint32_t q, uint64_t x) {
  uint32_t* size = &c.q.rings[q].tail.v;
  const uint32_t cap = (1u << c.q.nb_log2) - 1u;
  const uint32_t tgt = uni(ld32(size)) + 1u;
  if (tgt > cap) {
    pq_release(pq_lock(c, q, 1));
    fail(c, kStCapacity);
    return;
  }
  if (lane() == 0) {
    st32(size, tgt);
    st32(pq_state(c, q, tgt), tgt == 1u ? kNodeFull : kNodeTarget);
  }
  uint32_t i = 1;
  for (;;) {
    if (i == tgt) {
      pq_store(c, q, i, x);
      vm_drain();
      if (lane() == 0) st32(pq_state(c, q, i), kNodeFull);
      pq_release(pq_lock(c, q, i));
      return;
    }
    uint64_t lo, hi;
    merge64(pq_load(c, q, i), x, lo, hi);
    pq_store(c, q, i, lo);
    x = hi;
    // the child of i on the path to tgt
    const uint32_t below = (31u - (uint32_t)__clz(tgt)) - (31u - (uint32_t)__clz(i));
    const uint32_t next = tgt >> (below - 1u);
    if (!pq_acquire(c, pq_lock(c, q, next))) return;
    pq_release(pq_lock(c, q, i));
    i = next;
  }
}

// L2 Write to the priority queues.
__device__ __forceinline__ void pq_write(Ctx& c, uint64_t e, bool ok) {
  const uint32_t k = popc(ballot(ok));
  if (!k) return;
  const uint64_t x = sort64(ok ? e : kKeyInf);
  const uint32_t q = c.wq;
  c.wq = c.wq + 1u == c.q.nrings ? 0u : c.wq + 1u;
  if (lane() == 0) add32(&c.q.ctrl->pq_in.v, k);  // reserved before it can be read
  if (!pq_acquire(c, pq_lock(c, q, 1))) return;
  const uint32_t p = uni(ld32(pq_state(c, q, 0)));
  const uint64_t part = lane() < p ? pq_load(c, q, 0) : kKeyInf;
  uint64_t lo, hi;
  merge64(part, x, lo, hi);
  const uint32_t t = p + k;
  if (t < 64u) {
    if (lane() < t) pq_store(c, q, 0, lo);
    vm_drain();
    if (lane() == 0) st32(pq_state(c, q, 0), t);
    pq_release(pq_lock(c, q, 1));
    return;
  }
  if (lane() < t - 64u) pq_store(c, q, 0, hi);
  vm_drain();
  if (lane() == 0) st32(pq_state(c, q, 0), t - 64u);
  pq_push_full(c, q, lo);
  c.ct[kCtL2Writes] += 1;
}

// Takes up to 64 of the smallest elements of queue q (false: it was empty).
__device__ __forceinline__ bool pq_pop(Ctx& c, uint32_t q, uint64_t& e, bool& ok) {
  // a cheap look before taking the root lock
  const uint32_t size0 = uni(ld32(&c.q.rings[q].tail.v));
  const uint32_t p0 = uni(ld32(pq_state(c, q, 0)));
  if (size0 == 0u && p0 == 0u) return false;
  // a reader that finds the root busy for a while moves on (another queue,
  // or an idle turn) instead of queueing behind the writers
  if (!pq_acquire(c, pq_lock(c, q, 1), 6u)) return false;
  uint32_t* size = &c.q.rings[q].tail.v;
  const uint32_t n = uni(ld32(size));
  const uint32_t p = uni(ld32(pq_state(c, q, 0)));
  const uint64_t part = lane() < p ? pq_load(c, q, 0) : kKeyInf;
  if (n == 0u) {
    if (lane() == 0) st32(pq_state(c, q, 0), 0u);
    pq_release(pq_lock(c, q, 1));
    ok = lane() < p;
    e = part;
    return p != 0u;
  }
  uint64_t lo, hi;
  merge64(pq_load(c, q, 1), part, lo, hi);
  e = lo;
  ok = true;
  if (lane() < p) pq_store(c, q, 0, hi);
  if (n == 1u) {
    if (lane() == 0) {
      st32(size, 0u);
      st32(pq_state(c, q, 1), kNodeEmpty);
    }
    pq_release(pq_lock(c, q, 1));
    return true;
  }
  // wait, holding the root, until an insertion on its way to the last node
  // has arrived there, then move that node's batch to the root
  for (uint32_t spins = 0; uni(ld32(pq_state(c, q, n))) != kNodeFull; ++spins) {
    if ((spins & 63u) == 63u && must_stop(c)) {
      c.stop = true;
      return true;  // the query is over; the elements are never counted done
    }
    __builtin_amdgcn_s_sleep(1);
  }
  if (!pq_acquire(c, pq_lock(c, q, n))) return true;
  const uint64_t last = pq_load(c, q, n);
  if (lane() == 0) st32(pq_state(c, q, n), kNodeEmpty);
  pq_release(pq_lock(c, q, n));
  if (lane() == 0) st32(size, n - 1u);
  pq_store(c, q, 1, last);
  pq_sink(c, q, 1, last);
  c.ct[kCtL2Reads] += 1;
  return true;
}

// L2 Read from the priority queues: the wave's reading queue, then the others.
__device__ __forceinline__ bool pq_read(Ctx& c, uint64_t& e, bool& ok) {
  const uint32_t nq = c.q.nrings;
  for (uint32_t j = 0; j < nq && !c.stop; ++j) {
    const uint32_t q = c.rq + j < nq ? c.rq + j : c.rq + j - nq;
    if (pq_pop(c, q, e, ok)) return !c.stop;
  }
  return false;
}

// Ring of absolute bucket b seen from head bucket cur: bucket index relative
// to the head, clamped into [0, bmax - 1] (Section 4.2, L2DQ).
__device__ __forceinline__ uint32_t bucket_ring(const Ctx& c, uint32_t cur, uint32_t b) {
  const uint32_t nr = c.q.nrings;
  const uint32_t rel = b <= cur ? 0u : min(b - cur, nr - 1u);
  return (cur + rel) & (nr - 1u);
}

// Writes a vector to the bucket rings, one block per bucket present in it.
__device__ __forceinline__ void l2_write_direct(Ctx& c, uint32_t cur, uint64_t e, bool ok) {
  const uint32_t ring = bucket_ring(c, cur, elem_d(e) >> c.q.d2_log2);
  uint64_t m = ballot(ok);
  while (m) {
    const uint32_t r0 = lane_val(ring, first_lane(m));
    const bool sel = ok && ring == r0;
    const uint64_t ms = ballot(sel);
    if (!l2_put_block(c, r0, e, sel, ms)) return;
    ok = ok && !sel;
    m &= ~ms;
  }
}

// Write combining for the bucket queue: elements of the kStageB buckets after
// the head gather in one LDS row per bucket and go out as full 64-element
// blocks; the head bucket and farther buckets go out at once. A wave empties
// its rows whenever its L0 and L1 are empty, before it can count itself idle,
// so delayed-count termination still sees every element.
__device__ __forceinline__ void stage_flush_row(Ctx& c, uint32_t s, uint32_t cur) {
  const uint32_t n = lane_val(c.sn, s);
  const uint32_t b = lane_val(c.sb, s);
  if (n) {
    const bool ok = lane() < n;
    const uint64_t x = ok ? c.stage[s * 64u + lane()] : 0;
    compiler_fence();
    l2_put_block(c, bucket_ring(c, cur, b), x, ok, ballot(ok));
  }
  if (lane() == s) {
    c.sn = 0;
    c.sb = kInf;
  }
}

__device__ __forceinline__ void stage_flush_all(Ctx& c) {
  const uint64_t m = ballot(lane() < kStageB && c.sn != 0);
  if (!m) return;
  const uint32_t cur = uni(ld32(&c.q.ctrl->cur.v));
  for (uint64_t x = m; x && !c.stop; x &= x - 1) stage_flush_row(c, first_lane(x), cur);
}

// L2 Write of a lane vector.
__device__ __forceinline__ void l2_write(Ctx& c, uint64_t e, bool ok) {
  if (!ballot(ok)) return;
  if (c.pq) {
    pq_write(c, e, ok);
    return;
  }
  if (c.q.nrings == 1) {
    l2_put_block(c, 0, e, ok, ballot(ok));
    return;
  }
  const uint32_t cur = uni(ld32(&c.q.ctrl->cur.v));
  const uint32_t b = elem_d(e) >> c.q.d2_log2;
  const uint32_t window = min(kStageB, c.q.nrings - 1u);
  const bool st = c.stage != nullptr && ok && b > cur && b - cur <= window;
  const bool direct = ok && !st;
  if (ballot(direct)) l2_write_direct(c, cur, e, direct);
  // the window's buckets are consecutive, so each maps to its own row
  const uint32_t slot = b & (kStageB - 1u);
  uint64_t msk = ballot(st);
  while (msk && !c.stop) {
    const uint32_t f = first_lane(msk);
    const uint32_t s = lane_val(slot, f);
    const uint32_t bs = lane_val(b, f);
    const bool sel = st && slot == s;
    const uint64_t ms = ballot(sel);
    msk &= ~ms;
    if (lane_val(c.sb, s) != bs) {
      stage_flush_row(c, s, cur);  // the row held an older bucket
      if (lane() == s) c.sb = bs;
    }
    uint32_t cnt = lane_val(c.sn, s);
    const uint32_t k = popc(ms);
    const uint32_t r = rank_of(ms);
    const uint32_t room = 64u - cnt;
    if (sel && r < room) c.stage[s * 64u + cnt + r] = e;
    compiler_fence();
    if (k >= room) {
      // the row is full: it goes out as one block, the rest starts it anew
      if (lane() == s) c.sn = 64u;
      stage_flush_row(c, s, cur);
      if (lane() == s) c.sb = bs;
      if (sel && r >= room) c.stage[s * 64u + (r - room)] = e;
      compiler_fence();
      cnt = k - room;
    } else {
      cnt += k;
    }
    if (lane() == s) c.sn = cnt;
  }
}

// Take the block of ticket t of ring `ring` if it is published.
__device__ __forceinline__ bool l2_take(Ctx& c, uint32_t ring, uint32_t t, uint64_t& e, bool& ok) {
  const uint32_t nb = c.q.nb_log2;
  const uint32_t slot = t & ((1u << nb) - 1u);
  const uint32_t lap = t >> nb;
  const uint64_t bidx = ((uint64_t)ring << nb) + slot;
  uint64_t* h = c.q.hdr + bidx;
  const uint64_t hv = uni64(ld64(h));
  if ((uint32_t)(hv >> 32) != 2u * lap + 1u) return false;
  const uint32_t k = (uint32_t)hv;
  compiler_fence();
  ok = lane() < k;
  e = ok ? ld64(c.q.data + (bidx << 6) + lane()) : 0;
  vm_drain();
  if (lane() == 0) st64(h, (uint64_t)(2u * lap + 2u) << 32);
  c.ct[kCtL2Reads] += 1;
  return true;
}

// Read from one ring: keep a claimed ticket across READ_EMPTY (Section 4.2),
// else claim the oldest unread one. With few blocks available the claim is a
// compare-and-swap that never overshoots the writers; with many it is one
// atomicAdd (thousands of waves compare-and-swapping one counter serialise),
// whose rare overshoot leaves a pending claim that a later write fills.
__device__ __forceinline__ bool l2_try_ring(Ctx& c, uint32_t ring, uint32_t t_seen, uint32_t h_seen, uint64_t& e,
                                            bool& ok) {
  uint32_t p = lane_val(c.pend, ring);
  if (p == kInf) {
    RingCtr* rc = c.q.rings + ring;
    uint32_t claimed = 0;
    if (lane() == 0) {
      if ((int32_t)(t_seen - h_seen) > 64) {
        p = add32(&rc->head.v, 1u);
        claimed = 1;
      } else {
        uint32_t h = h_seen;
        for (int i = 0; i < 4 && (int32_t)(t_seen - h) > 0; ++i) {
          if (cas32(&rc->head.v, h, h + 1u)) {
            p = h;
            claimed = 1;
            break;
          }
          h = ld32(&rc->head.v);
          t_seen = ld32(&rc->tail.v);
        }
      }
    }
    if (!lane_val(claimed, 0)) return false;
    p = lane_val(p, 0);
  }
  for (int i = 0; i < 4; ++i) {
    if (l2_take(c, ring, p, e, ok)) {
      if (lane() == ring) c.pend = kInf;
      return true;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  if (lane() == ring) c.pend = p;
  return false;
}

// The bucket rings form a calendar: a ring read as bucket cur + j may still
// hold elements of a later lap (written when it was the catch-all last
// bucket). Those go back to the bucket they belong to now instead of being
// expanded ahead of the frontier.
__device__ __forceinline__ void defer_later(Ctx& c, uint32_t cur, uint32_t j, uint64_t e, bool& ok) {
  const uint32_t b = elem_d(e) >> c.q.d2_log2;
  const uint32_t rel = b <= cur ? 0u : min(b - cur, c.q.nrings - 1u);
  const bool later = ok && rel > j;
  if (ballot(later)) {
    l2_write(c, e, later);
    ok = ok && !later;
  }
}

// L2 Read.
__device__ __forceinline__ bool l2_read(Ctx& c, uint64_t& e, bool& ok) {
  if (c.pq) return pq_read(c, e, ok);
  if (c.q.nrings == 1) {
    uint32_t t = 0, h = 0;
    if (lane_val(c.pend, 0) == kInf) {
      const uint32_t credit = lane_val(c.pend, 1);
      if (credit != kInf && credit != 0u) {
        // the ring held many blocks when last read: claim by atomicAdd at
        // once, one memory round trip fewer (an overshoot is a pending claim
        // that a later write fills, as on the atomicAdd path below)
        if (lane() == 1) c.pend = credit - 1u;
        t = 65u;
        h = 0u;
      } else {
        t = uni(ld32(&c.q.rings[0].tail.v));
        h = uni(ld32(&c.q.rings[0].head.v));
        if ((int32_t)(t - h) <= 0) return false;
        // a few claims without looking, if the backlog dwarfs them
        if (lane() == 1) c.pend = (int32_t)(t - h) > 1024 ? 3u : kInf;
      }
    }
    return l2_try_ring(c, 0, t, h, e, ok);
  }
  // Bucket queue.
  const uint32_t nr = c.q.nrings;
  const uint32_t cur = uni(ld32(&c.q.ctrl->cur.v));
  // Blocks this wave already claimed are taken first, wherever their rings
  // now sit in the calendar. A claim whose block is not written yet does not
  // stop the wave from reading other rings: if every wave waited on such a
  // claim, nobody would produce the writes that fill them.
  const uint64_t pm = ballot(lane() < nr && c.pend != kInf);
  for (uint64_t mp = pm; mp;) {
    const uint32_t r = first_lane(mp);
    mp &= mp - 1;
    if (l2_try_ring(c, r, 0, 0, e, ok)) {
      defer_later(c, cur, (r - cur) & (nr - 1u), e, ok);
      return true;
    }
  }
  // lane i looks at bucket cur + i
  const bool in = lane() < nr;
  const uint32_t r = (cur + lane()) & (nr - 1u);
  uint32_t t = 0, h = 0;
  if (in) {
    t = ld32(&c.q.rings[r].tail.v);
    h = ld32(&c.q.rings[r].head.v);
  }
  const uint64_t m = ballot(in && (int32_t)(t - h) > 0);
  // The base moves to the first non-empty bucket once the head bucket is
  // empty and no wave holds work in its own L0/L1 (all are idle): work held
  // privately is part of the head bucket too, and moving on without it lets
  // the grid run ahead of the frontier. A wave that has found nothing for a
  // while moves it anyway, which bounds the wait when local queues stay busy.
  if (m && !(m & 1u)) {
    bool go = c.idle >= 8u;
    if (!go) {
      const uint32_t hungry = uni(ld32(&c.q.ctrl->hungry.v));
      const uint32_t act = uni(ld32(&c.q.ctrl->active.v));
      go = hungry >= act;
    }
    if (go && lane() == 0) cas32(&c.q.ctrl->cur.v, cur, cur + first_lane(m));
  }
  // rings where this wave already holds a claim were tried above
  const uint32_t pend_r = __shfl(c.pend, (int)r);
  const uint64_t busy = ballot(in && pend_r != kInf);
  uint64_t mw = m & ~busy & (c.q.bnum >= 64 ? ~0ull : ((1ull << c.q.bnum) - 1ull));
  while (mw) {
    const uint32_t j = first_lane(mw);
    mw &= mw - 1;
    if (l2_try_ring(c, (cur + j) & (nr - 1u), lane_val(t, j), lane_val(h, j), e, ok)) {
      defer_later(c, cur, j, e, ok);
      return true;
    }
  }
  return false;
}

// ------------------------------------------------------------ grid-wide hub tier

// A vertex of very high degree is not expanded by one wave: its edge range is
// published as a record whose chunks any wave of the grid can claim.
__device__ __forceinline__ void hub_post(Ctx& c, bool p, uint32_t v, uint32_t d, uint32_t beg, uint32_t end) {
  QueryCtrl* ctl = c.q.ctrl;
  const uint32_t ch = c.q.hub_chunk;
  uint32_t r = kInf;
  if (p) {
    add32(&ctl->hub_units.v, (end - beg + ch - 1u) / ch);  // reserve before publishing
    r = add32(&ctl->hub_tail.v, 1u);
    if (r < c.q.hub_cap) {
      st64(c.q.hub_rec + 2ull * r, make_elem(v, d));
      st64(c.q.hub_rec + 2ull * r + 1, (uint64_t)beg | ((uint64_t)end << 32));
    }
  }
  vm_drain();
  if (p && r < c.q.hub_cap) st32(c.q.hub_pub + r, 1u);
  if (ballot(p && r >= c.q.hub_cap)) fail(c, kStHubCapacity);
}

__device__ __forceinline__ bool hub_claim(Ctx& c, uint32_t& v, uint32_t& d, uint32_t& eb, uint32_t& ee) {
  if (!c.q.th_hub) return false;
  QueryCtrl* ctl = c.q.ctrl;
  const uint32_t h = uni(ld32(&ctl->hub_head.v));
  const uint32_t t = min(uni(ld32(&ctl->hub_tail.v)), c.q.hub_cap);
  const uint32_t ch = c.q.hub_chunk;
  for (uint32_t r = h; r < t && r < h + 8u; ++r) {
    if (uni(ld32(c.q.hub_pub + r)) == 0) continue;
    const uint64_t x0 = uni64(ld64(c.q.hub_rec + 2ull * r));
    const uint64_t x1 = uni64(ld64(c.q.hub_rec + 2ull * r + 1));
    const uint32_t beg = (uint32_t)x1, end = (uint32_t)(x1 >> 32);
    const uint32_t nch = (end - beg + ch - 1u) / ch;
    uint32_t ci = 0;
    if (lane() == 0) ci = add32(c.q.hub_cur + r, 1u);
    ci = lane_val(ci, 0);
    if (ci < nch) {
      v = elem_v(x0);
      d = elem_d(x0);
      eb = beg + ci * ch;
      ee = min(end, eb + ch);
      if (ci + 1u == nch && lane() == 0) cas32(&ctl->hub_head.v, r, r + 1u);
      return true;
    }
    if (lane() == 0) cas32(&ctl->hub_head.v, r, r + 1u);
  }
  return false;
}

// ------------------------------------------------------------ L1 (LDS, private to the wave)

// Near-far re-split (Section 3.4, L1NF): when near is empty, NF = min(far) +
// delta1 and far elements below NF move to near; the rest is compacted in place.
__device__ __forceinline__ void nf_resplit(Ctx& c) {
  const uint32_t fh = c.fh, ft = c.ft;
  const uint32_t cnt = ft - fh;
  uint32_t mn = kInf;
  for (uint32_t j = lane(); j < cnt; j += 64) mn = min(mn, elem_d(c.far[(fh + j) & c.l1mask]));
  mn = uni(wave_min(mn));
  const uint32_t nf = sat_add(mn, c.q.delta1);
  uint32_t qt = c.qt, wp = fh;
  for (uint32_t j = 0; j < cnt; j += 64) {
    const bool has = j + lane() < cnt;
    const uint64_t x = has ? c.far[(fh + j + lane()) & c.l1mask] : 0;
    compiler_fence();
    const bool tonear = has && elem_d(x) < nf;
    const bool keep = has && !tonear;
    const uint64_t m1 = ballot(tonear), m2 = ballot(keep);
    if (tonear) c.l1[(qt + rank_of(m1)) & c.l1mask] = x;
    if (keep) c.far[(wp + rank_of(m2)) & c.l1mask] = x;
    compiler_fence();
    qt += popc(m1);
    wp += popc(m2);
  }
  c.thresh = nf;
  c.qt = qt;
  c.ft = wp;
}

__device__ __forceinline__ bool l1_empty(const Ctx& c) { return c.qh == c.qt && c.fh == c.ft; }

// L1 Read: up to 64 elements, near ring first.
__device__ __forceinline__ bool l1_take(Ctx& c, uint64_t& e, bool& ok) {
  if (c.q.l1_type == MLMQ_L1_NEARFAR && c.qt == c.qh && c.ft != c.fh) nf_resplit(c);
  const uint32_t k = min(c.qt - c.qh, 64u);
  ok = lane() < k;
  e = ok ? c.l1[(c.qh + lane()) & c.l1mask] : 0;
  compiler_fence();
  c.qh += k;
  return k != 0;
}

// L1 Write. Lanes that must go to L2 come back in `spill`.
// Returns true when an L1V periodic flush is due.
__device__ __forceinline__ bool l1_put(Ctx& c, uint64_t e, bool ok, bool& spill) {
  const uint32_t cap = c.q.l1_cap;
  const uint32_t d = elem_d(e);
  if (c.q.l1_type == MLMQ_L1_NEARFAR) {
    const bool np = ok && d < c.thresh;
    const bool fp = ok && !np;
    const uint64_t mn = ballot(np), mf = ballot(fp);
    const uint32_t sn = cap - (c.qt - c.qh), sf = cap - (c.ft - c.fh);
    const uint32_t rn = rank_of(mn), rf = rank_of(mf);
    if (np && rn < sn) c.l1[(c.qt + rn) & c.l1mask] = e;
    if (fp && rf < sf) c.far[(c.ft + rf) & c.l1mask] = e;
    compiler_fence();
    spill = (np && rn >= sn) || (fp && rf >= sf);
    c.qt += min(popc(mn), sn);
    c.ft += min(popc(mf), sf);
    return false;
  }
  if (c.q.l1_type == MLMQ_L1_SLF) {
    // Small-Label-First deque (Section 3.4): items shorter than the head go
    // in front of it (read next), the others at the back.
    const uint32_t hd = c.qt != c.qh ? elem_d(c.l1[c.qh & c.l1mask]) : kInf;
    compiler_fence();
    const bool fr = ok && d < hd;
    const bool bk = ok && !fr;
    const uint64_t mf = ballot(fr), mb = ballot(bk);
    uint32_t space = cap - (c.qt - c.qh);
    const uint32_t nf = min(popc(mf), space);
    const uint32_t rf = rank_of(mf);
    if (fr && rf < nf) c.l1[(c.qh - nf + rf) & c.l1mask] = e;
    space -= nf;
    const uint32_t nb = min(popc(mb), space);
    const uint32_t rb = rank_of(mb);
    if (bk && rb < nb) c.l1[(c.qt + rb) & c.l1mask] = e;
    compiler_fence();
    spill = (fr && rf >= nf) || (bk && rb >= nb);
    c.qh -= nf;
    c.qt += nb;
    return false;
  }
  bool keep = ok;
  spill = false;
  if (c.q.l1_type == MLMQ_L1_FILTER) {
    keep = ok && d <= c.thresh;
    spill = ok && !keep;
  }
  const uint64_t m = ballot(keep);
  const uint32_t space = cap - (c.qt - c.qh);
  const uint32_t r = rank_of(m);
  if (keep && r < space) c.l1[(c.qt + r) & c.l1mask] = e;
  compiler_fence();
  spill = spill || (keep && r >= space);
  c.qt += min(popc(m), space);
  if (c.q.l1_type == MLMQ_L1_VEC && c.q.l1_wb) {
    if (++c.wcount >= c.q.l1_wb) {
      c.wcount = 0;
      return true;
    }
  }
  return false;
}

// L1V periodic flush: everything currently in L1 goes back to L2.
__device__ __forceinline__ void l1_flush(Ctx& c) {
  c.ct[kCtFlushes] += 1;
  while (c.qt != c.qh && !c.stop) {
    uint64_t x = 0;
    bool ok = false;
    l1_take(c, x, ok);
    l2_write(c, x, ok);
  }
}

// Write cascade below L0: L1, whose overflow goes to L2.
__device__ __forceinline__ void write_l1(Ctx& c, uint64_t e, bool ok) {
  if (c.q.l1_type == MLMQ_L1_NONE) {
    l2_write(c, e, ok);
    return;
  }
  bool spill = false;
  const bool flush = l1_put(c, e, ok, spill);
  c.ct[kCtL1Writes] += 1;
  if (ballot(spill)) l2_write(c, e, spill);
  if (flush) l1_flush(c);
}

// Work sharing between the levels: while other waves of the query find no
// work, a wave whose L1 main (near) ring holds at least donate_min elements hands the
// older half of it to L2, where the idle waves pick it up; the far ring stays
// private, since handing it out would put work ahead of the frontier. Without
// this a wave can keep a whole wavefront in its private L1 (the near-far and
// filter queues never overflow on low-degree graphs) while the grid waits.
__device__ __forceinline__ void donate(Ctx& c) {
  uint32_t give = (c.qt - c.qh) / 2u;
  c.ct[kCtDonations] += 1;
  while (give && !c.stop) {
    const uint32_t k = min(give, 64u);
    const bool ok = lane() < k;
    const uint64_t x = ok ? c.l1[(c.qh + lane()) & c.l1mask] : 0;
    compiler_fence();
    c.qh += k;
    give -= k;
    l2_write(c, x, ok);
  }
}

// L0 full: all of its elements move to L1 (Section 3.4, L0 queue).
__device__ __forceinline__ void spill_l0(Ctx& c) {
  while (c.l0n && !c.stop) {
    uint64_t x;
    bool ok;
    l0_read(c, x, ok);
    write_l1(c, x, ok);
  }
}

// Unified Write of the lanes' new work items (after wave compaction).
__device__ __forceinline__ void emit(Ctx& c, uint32_t v, uint32_t nd, bool imp) {
  const uint64_t m = ballot(imp);
  if (!m) return;
  const uint32_t k = popc(m);
  c.ct[kCtPushes] += k;
  const uint64_t e = make_elem(v, nd);
  if (c.q.l0_cap) {
    if (c.l0n + k > c.q.l0_cap) spill_l0(c);
    stage(c, e, imp);
    l0_append(c, k);
  } else {
    write_l1(c, e, imp);
  }
}

// ------------------------------------------------------------ relaxation

// Edges a lane relaxes per step: the loads of all of them are issued before
// any result is used, so a wave has kRelaxUnroll independent memory chains
// in flight instead of one.
constexpr int kRelaxUnroll = 4;

// Relax U sub-batches of 64 edges, given as packed edge words (one edge per
// lane each; the relax step of the paper's kernel sketch, with atomicMin):
// candidate nd = d + w
// (saturating), a plain load of dist[v] filters hopeless candidates (unless
// the query relaxes by atomicMin alone), then atomicMin decides; a lane has
// new work iff nd < the previous label.
// Lanes without a candidate load the label of vertex 0 (and, in relax_many,
// edge word 0): both exist whenever there is an edge to relax, so every load
// is unconditional.
template <int U>
__device__ __forceinline__ void relax_words(Ctx& c, const bool (&has)[U], const uint64_t (&a)[U],
                                            const uint32_t (&d)[U]) {
  uint32_t v[U], nd[U], lab[U];
  bool cand[U];
  bool of = false;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint64_t sum = (uint64_t)d[u] + (c.q.unit_w ? 1ull : (a[u] >> 32));
    of = of || (has[u] && sum >= kInf);
    cand[u] = has[u] && sum < kInf;
    v[u] = (uint32_t)a[u];
    nd[u] = (uint32_t)sum;
    const uint32_t lv = cand[u] ? v[u] : 0u;
    lab[u] = c.q.relax_mode == MLMQ_RELAX_ATOMIC ? kInf : ld_label(c.q.dist + lv);
  }
  bool imp[U];
  uint32_t natom = 0;
#pragma unroll
  for (int u = 0; u < U; ++u) natom += popc(ballot(cand[u] && nd[u] < lab[u]));
  c.ct[kCtAtomics] += natom;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    imp[u] = false;
    if (cand[u] && nd[u] < lab[u]) {
      const uint32_t old =
          __hip_atomic_fetch_min(c.q.dist + v[u], nd[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      imp[u] = nd[u] < old;
    }
  }
  uint32_t nedges = 0;
#pragma unroll
  for (int u = 0; u < U; ++u) nedges += popc(ballot(has[u]));
  c.ct[kCtEdges] += nedges;
  if (ballot(of)) c.ovf = true;
#pragma unroll
  for (int u = 0; u < U; ++u) emit(c, v[u], nd[u], imp[u]);
}

// The same for edges given by their CSR positions: the packed edge words are
// loaded first.
template <int U>
__device__ __forceinline__ void relax_many(Ctx& c, const bool (&has)[U], const uint32_t (&ed)[U],
                                           const uint32_t (&d)[U]) {
  uint64_t a[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint32_t eidx = has[u] ? ed[u] : 0u;
    a[u] = c.q.adj[eidx];
  }
  relax_words<U>(c, has, a, d);
}

// Whole wave sweeps the edge range [eb, ee) of vertex v at distance d. Every
// 1024 edges it looks at dist[v] again (the load goes out with that step's
// label loads and is read after it): once v has been improved, the rest of
// the sweep is redundant (the improved item expands all of it anyway).
__device__ __forceinline__ void process_range(Ctx& c, uint32_t v, uint32_t d, uint32_t eb, uint32_t ee) {
  constexpr int U = kRelaxUnroll;
  uint32_t x = eb;
  if (x + 64u * U <= ee && !c.stop) {
    // the edge words of the next step are loaded before the current step is
    // relaxed, so their latency overlaps the label loads and atomics
    uint64_t nx[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t eidx = x + 64u * u + lane();
      nx[u] = c.q.adj[eidx];
    }
    for (;;) {
      uint64_t a[U];
#pragma unroll
      for (int u = 0; u < U; ++u) a[u] = nx[u];
      const uint32_t xn = x + 64u * U;
      const bool more = xn + 64u * U <= ee;
      if (more) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t eidx = xn + 64u * u + lane();
          nx[u] = c.q.adj[eidx];
        }
      }
      const bool chk = x != eb && ((x - eb) & 1023u) == 0;
      const uint32_t cur = chk ? ld_label(c.q.dist + v) : kInf;
      bool has[U];
      uint32_t dd[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        has[u] = true;
        dd[u] = d;
      }
      relax_words<U>(c, has, a, dd);
      x = xn;
      if (!more || c.stop) break;
      if (chk && uni(cur) < d) return;
    }
  }
  for (; x < ee && !c.stop; x += 64) {
    bool has[1] = {x + lane() < ee};
    uint32_t ed[1] = {x + lane()}, dd[1] = {d};
    relax_many<1>(c, has, ed, dd);
  }
}

// Edge idx of the flattened batch: lane j owns edges [excl_j, incl_j) of the
// batch, starting at CSR position beg_j; binary search over the inclusive scan.
__device__ __forceinline__ void flat_edge(uint32_t idx, uint32_t incl, uint32_t excl, uint32_t beg, uint32_t d,
                                          uint32_t& ed, uint32_t& dd) {
  uint32_t j = 0;
#pragma unroll
  for (uint32_t st = 32; st; st >>= 1) {
    if ((uint32_t)__shfl(incl, (int)(j + st - 1)) <= idx) j += st;
  }
  ed = (uint32_t)__shfl(beg, (int)j) + (idx - (uint32_t)__shfl(excl, (int)j));
  dd = (uint32_t)__shfl(d, (int)j);
}

// Relaxation of a batch (the paper's SSSP_relax with the load balancing of
// Section 4.1): drop stale items, send very-high-degree vertices to the
// grid-wide tier, let the whole wave sweep vertices above th_v, and spread the
// edges of the remaining vertices evenly over the lanes.
__device__ __forceinline__ void process_vec(Ctx& c, uint64_t e, bool ok) {
  const uint32_t v = elem_v(e), d = elem_d(e);
  // label and row bounds are loaded together (vertex 0 for idle lanes)
  const uint32_t lv = ok ? v : 0u;
  const uint32_t label = ld_label(c.q.dist + lv);
  const uint32_t beg0 = (uint32_t)c.q.off[lv];
  const uint32_t end0 = (uint32_t)c.q.off[lv + 1];
  const bool stale = ok && d > label;
  c.ct[kCtStale] += popc(ballot(stale));
  ok = ok && !stale;
  c.ct[kCtExpansions] += popc(ballot(ok));
  const uint32_t beg = ok ? beg0 : 0u, end = ok ? end0 : 0u;
  const uint32_t deg = end - beg;
  if (c.q.th_hub) {
    const bool hub = ok && deg > c.q.th_hub;
    if (ballot(hub)) {
      hub_post(c, hub, v, d, beg, end);
      ok = ok && !hub;
      if (c.stop) return;
    }
  }
  const bool big = ok && deg > c.q.th_v;
  const uint32_t sdeg = (ok && !big) ? deg : 0u;
  const uint32_t incl = wave_incl_scan(sdeg);
  const uint32_t total = lane_val(incl, 63);
  const uint32_t excl = incl - sdeg;
  constexpr int U = kRelaxUnroll;
  uint32_t base = 0;
  for (; base + 64u * (U - 1) < total && !c.stop; base += 64u * U) {
    bool has[U];
    uint32_t ed[U], dd[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t idx = base + 64u * u + lane();
      has[u] = idx < total;
      flat_edge(has[u] ? idx : 0u, incl, excl, beg, d, ed[u], dd[u]);
    }
    relax_many<U>(c, has, ed, dd);
  }
  for (; base < total && !c.stop; base += 64) {
    const uint32_t idx = base + lane();
    bool has[1] = {idx < total};
    uint32_t ed[1], dd[1];
    flat_edge(has[0] ? idx : 0u, incl, excl, beg, d, ed[0], dd[0]);
    relax_many<1>(c, has, ed, dd);
  }
  uint64_t mb = ballot(big);
  while (mb && !c.stop) {
    const uint32_t j = first_lane(mb);
    mb &= mb - 1;
    process_range(c, lane_val(v, j), lane_val(d, j), lane_val(beg, j), lane_val(end, j));
  }
}

// ------------------------------------------------------------ termination

// Delayed-count emptiness test (Section 4.1): read done first, then the
// reservations; equality means no work existed when done was read.
__device__ __forceinline__ bool try_terminate(Ctx& c) {
  QueryCtrl* ctl = c.q.ctrl;
  const uint32_t done = uni(ld32(&ctl->done.v));
  vm_drain();
  // reservations: ring tickets (blocks), or elements written to the priority queues
  const uint32_t t = c.pq ? (lane() == 0 ? ld32(&ctl->pq_in.v) : 0u)
                          : (lane() < c.q.nrings ? ld32(&c.q.rings[lane()].tail.v) : 0u);
  const uint32_t units = c.q.th_hub ? uni(ld32(&ctl->hub_units.v)) : 0u;
  const uint32_t reserved = uni(wave_sum(t)) + units;
  if (done == reserved) {
    if (lane() == 0) st32(&ctl->terminate.v, 1u);
    return true;
  }
  return false;
}

// Threshold of the filter queue after taking a batch whose smallest distance
// is mn (our reading: F = min + delta1 on every refill from the global levels).
__device__ __forceinline__ void refill_threshold(Ctx& c, uint32_t mn) {
  if (c.q.l1_type == MLMQ_L1_FILTER) c.thresh = sat_add(mn, c.q.delta1);
}

// Keeps ctrl->hungry equal to the number of this query's waves that found
// no work on their last look.
__device__ __forceinline__ void set_hungry(Ctx& c, bool h) {
  if (c.hungry == h) return;
  c.hungry = h;
  if (lane() == 0) add32(&c.q.ctrl->hungry.v, h ? 1u : 0xFFFFFFFFu);
}

// The persistent worker loop of one wave on one query (the paper's work
// kernel with the manager's emptiness test folded in).
__device__ __forceinline__ void run_query(Ctx& c) {
  const uint64_t t_start = (uint64_t)wall_clock64();
  uint64_t t_idle = 0;
  if (lane() == 0) add32(&c.q.ctrl->active.v, 1u);
  while (!c.stop) {
    ++c.it;
    beat_loop(c.beat, kPtLoop, c.it);
    if ((c.it & 63u) == 0 && must_stop(c)) break;
    uint64_t e = 0;
    bool ok = false, got = false;
    if (c.l0n) {
      l0_read(c, e, ok);
      got = true;
    } else if (c.q.l1_type != MLMQ_L1_NONE && !l1_empty(c)) {
      // looked at on every take while the ring is long enough to share: on
      // grids the idle waves get work a few microseconds sooner (every 16th
      // take measured 10% slower on the 2048 x 2048 road-like grid). Over a
      // single heap only every 16th take: each donation is a block inserted
      // at the one root lock (road-like 512 x 512 grid: 78.5 ms against 144)
      if ((!c.pq || c.q.nrings > 1 || (c.it & 15u) == 0) && c.qt - c.qh >= c.q.donate_min &&
          uni(ld32(&c.q.ctrl->hungry.v)) != 0)
        donate(c);
      got = l1_take(c, e, ok);
      c.ct[kCtL1Reads] += 1;
    } else {
      if (c.stage) stage_flush_all(c);
      uint32_t hv, hd, heb, hee;
      beat_loop(c.beat, kPtHub, c.it);
      if (hub_claim(c, hv, hd, heb, hee)) {
        set_hungry(c, false);
        c.done_acc += 1u;
        refill_threshold(c, hd);
        c.ct[kCtHubChunks] += 1;
        c.idle = 0;
        if (hd <= uni(ld_label(c.q.dist + hv))) process_range(c, hv, hd, heb, hee);
        continue;
      }
      beat_loop(c.beat, kPtL2Read, c.it);
      got = l2_read(c, e, ok);
      if (got) {
        set_hungry(c, false);
        c.done_acc += c.pq ? popc(ballot(ok)) : 1u;  // elements (priority queues) or one block
        refill_threshold(c, uni(wave_min(ok ? elem_d(e) : kInf)));
      } else {
        // Idle: the wave holds nothing, so its delayed count can go out.
        beat_loop(c.beat, kPtIdle, c.it);
        const uint64_t t0 = (uint64_t)wall_clock64();
        if (c.done_acc) {
          uint32_t r = 0;
          if (lane() == 0) r = add32(&c.q.ctrl->done.v, c.done_acc);
          (void)lane_val(r, 0);
          vm_drain();
          c.done_acc = 0;
        }
        set_hungry(c, true);
        if (try_terminate(c)) break;
        if ((++c.idle & 7u) == 0 && must_stop(c)) break;
        backoff(min(c.idle >> 2, 6u));
        t_idle += (uint64_t)wall_clock64() - t0;
        continue;
      }
    }
    c.idle = 0;
    beat_loop(c.beat, kPtProcess, c.it);
    process_vec(c, e, ok);
  }
  set_hungry(c, false);
  if (lane() == 0) add32(&c.q.ctrl->active.v, 0xFFFFFFFFu);
  c.ct64_wave = (uint64_t)wall_clock64() - t_start;
  c.ct64_idle = t_idle;
  beat(c.beat, kPtDone, c.it);
}

// Next query for this wave: queries are taken in order; each accepts up to
// want_wgs workgroups over its lifetime.
__device__ __forceinline__ uint32_t pick_query(const LaunchArgs& a) {
  uint32_t q = kInf;
  if (lane() == 0 && ld32(&a.batch->cancel.v) == 0) {
    for (uint32_t i = ld32(&a.batch->cursor.v); i < (uint32_t)a.nq; ++i) {
      const QueryDesc* d = a.queries + i;
      if (ld32(&d->ctrl->terminate.v) == 0 && add32(&d->ctrl->joined.v, 1u) < d->want_wgs) {
        q = i;
        break;
      }
      cas32(&a.batch->cursor.v, i, i + 1);
    }
  }
  return lane_val(q, 0);
}

// ------------------------------------------------------------ kernels

// Fresh wave state for query q: empty L0 and L1 (the LDS rings need no
// clearing, only their counters), no pending tickets, no counters.
__device__ __forceinline__ void setup_ctx(Ctx& c, const QueryDesc& q, uint64_t* smem, uint32_t l1_cap_alloc,
                                          uint32_t two_alloc, uint32_t stage_alloc, const uint32_t* cancel,
                                          uint64_t deadline, uint64_t cap_wait, uint32_t* beat_word, bool pq_kernel) {
  c.q = q;
  // pq_kernel is a literal at each kernel, so the ring-only variant drops
  // every priority-queue branch; the host launches the priority-queue
  // variant whenever a query of the launch uses priority queues
  c.pq = pq_kernel && q.l2_type == MLMQ_L2_PQ;
  c.rq = c.pq ? blockIdx.x % q.nrings : 0u;
  c.wq = c.rq;
  c.stg = smem;
  c.l1 = smem + 64;
  c.far = c.l1 + l1_cap_alloc;
  c.stage = (stage_alloc && q.nrings > 1) ? c.far + (two_alloc ? l1_cap_alloc : 0u) : nullptr;
  c.sb = kInf;
  c.sn = 0;
  c.l1mask = c.q.l1_cap - 1u;
  c.qh = c.qt = c.fh = c.ft = 0;
  c.thresh = c.q.l1_type == MLMQ_L1_FILTER ? c.q.delta1 : 0u;
  c.wcount = 0;
  c.done_acc = 0;
  c.pend = kInf;
  c.cancel = cancel;
  c.deadline = deadline;
  c.cap_wait = cap_wait;
  c.r0 = c.r1 = c.r2 = c.r3 = 0;
  c.l0h = c.l0n = 0;
  c.beat = beat_word;
  c.it = 0;
  c.stop = false;
  c.ovf = false;
  c.hungry = false;
  c.idle = 0;
  c.ct64_wave = c.ct64_idle = 0;
#pragma unroll
  for (int i = 0; i < kNumCounters; ++i) c.ct[i] = 0;
}

// Adds this wave's counters and overflow flag to the query's control block.
__device__ __forceinline__ void flush_counters(const Ctx& c) {
  if (lane() == 0) {
    QueryCtrl* ctl = c.q.ctrl;
#pragma unroll
    for (int i = 0; i < kCtWaveTicks; ++i)
      if (c.ct[i]) __hip_atomic_fetch_add(&ctl->stats[i], (uint64_t)c.ct[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&ctl->stats[kCtWaveTicks], c.ct64_wave, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&ctl->stats[kCtIdleTicks], c.ct64_idle, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (c.ovf) st32(&ctl->overflow.v, 1u);
  }
}

// ---------------------------------------------------------------- server slots
//
// A server slot word packs (generation << 32) | closed << 31 | want << 16 |
// joined. The host opens a slot (closed = 0, joined = 0) once the query's
// memory is initialised. A wave that sees an open slot joins by one atomicAdd
// on the word: it is in iff the value it got back was open (whatever the
// generation: the descriptor is read after joining) with joined < want, so
// the waves that lose a race to a full or closed slot do not retry against
// each other (a CAS loop here made 2000 idle waves take turns on one word for
// tens of milliseconds). Their increments only count past want or after the
// close. The first wave to leave closes the slot; the waves on the query are
// then the min(joined, want) counted before the close, and that wave adds this
// number to the high half of the query's finished counter, so the wave whose
// increment makes the low half equal the high half is the last one out and
// reports completion to the host.

constexpr uint64_t kSlotClosed = 1ull << 31;
__device__ __forceinline__ uint32_t slot_gen(uint64_t w) { return (uint32_t)(w >> 32); }
__device__ __forceinline__ uint32_t slot_want(uint64_t w) { return (uint32_t)(w >> 16) & 0x7FFFu; }
__device__ __forceinline__ uint32_t slot_joined(uint64_t w) { return (uint32_t)w & 0xFFFFu; }
__device__ __forceinline__ bool slot_open(uint64_t w) {
  return slot_gen(w) != 0 && (w & kSlotClosed) == 0 && slot_joined(w) < slot_want(w);
}

// Loads a descriptor with coherent loads (lane i reads 8-byte word i): the
// slot table is rewritten while the kernel runs, so no cached copy may be used.
__device__ __forceinline__ QueryDesc load_desc_coherent(const QueryDesc* d) {
  static_assert(sizeof(QueryDesc) % 8 == 0 && sizeof(QueryDesc) / 8 <= 64, "descriptor layout");
  constexpr int kWords = sizeof(QueryDesc) / 8;
  const uint64_t mine = lane() < (uint32_t)kWords ? ld64(reinterpret_cast<const uint64_t*>(d) + lane()) : 0ull;
  uint64_t w[kWords];
#pragma unroll
  for (int i = 0; i < kWords; ++i) {
    const uint32_t lo = lane_val((uint32_t)mine, (uint32_t)i), hi = lane_val((uint32_t)(mine >> 32), (uint32_t)i);
    w[i] = (uint64_t)lo | ((uint64_t)hi << 32);
  }
  QueryDesc q;
  __builtin_memcpy(&q, w, sizeof(q));
  return q;
}

}  // namespace

// ------------------------------------------------------------ kernels

// One wave per workgroup; dynamic LDS = staging row + L1 ring(s). Three waves
// per SIMD are asked of the register allocator: the worker runs up to 12
// workgroups per CU (batches and the server fill the device), and the limit
// also measured faster at the default launch sizes.
template <bool kPQ>
__device__ __forceinline__ void worker_body(const LaunchArgs& a) {
  extern __shared__ uint64_t smem[];
  const uint64_t t0 = (uint64_t)wall_clock64();
  uint32_t* const my_beat = a.beats ? a.beats + blockIdx.x : nullptr;
  for (;;) {
    beat(my_beat, kPtPick, 0);
    const uint32_t qi = pick_query(a);
    if (qi == kInf) break;
    Ctx c;
    setup_ctx(c, a.queries[qi], smem, a.l1_cap, a.l1_two, a.stage, &a.batch->cancel.v, t0 + a.timeout_ticks,
              a.cap_wait_ticks, my_beat, kPQ);
    run_query(c);
    flush_counters(c);
    if (lane() == 0) add32(&c.q.ctrl->finished.v, 1u);
  }
}

__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) mlmq_worker(LaunchArgs a) {
  worker_body<false>(a);
}
// The same worker with the L2 priority-queue code compiled in.
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) mlmq_worker_pq(LaunchArgs a) {
  worker_body<true>(a);
}

// Resident server kernel: each wave repeatedly joins the oldest open slot,
// works on that query until it terminates, and leaves. Idle waves sleep and
// leave the kernel on the host's stop flag or after idle_exit_ticks without
// work (the host relaunches the kernel when work arrives and none is left).
template <bool kPQ>
__device__ __forceinline__ void server_body(const ServerArgs& a) {
  extern __shared__ uint64_t smem[];
  uint64_t last_busy = (uint64_t)wall_clock64();
  uint32_t idle = 0;
  for (;;) {
    const uint32_t l = lane();
    const uint64_t w = l < (uint32_t)a.nslots ? ld64(&a.join[l]) : 0ull;
    const bool open = slot_open(w);
    const uint32_t g = uni(wave_min(open ? slot_gen(w) : kInf));
    if (g != kInf) {
      const uint32_t s = first_lane(ballot(open && slot_gen(w) == g));
      uint32_t won = 0;
      if (l == 0) {
        const uint64_t got = __hip_atomic_fetch_add(&a.join[s], 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        won = slot_open(got) ? 1u : 0u;
      }
      if (!lane_val(won, 0)) {
        // lost the race: the slot filled or closed; look again after a pause
        ++idle;
        backoff(min(idle >> 2, 6u));
        continue;
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const uint32_t t_join = (uint32_t)wall_clock64();  // read by the whole wave
      if (l == 0) st32(&a.ctl->last_busy.v, t_join);
      const QueryDesc q = load_desc_coherent(a.slots + s);
      Ctx c;
      setup_ctx(c, q, smem, a.l1_cap, a.l1_two, a.stage, &a.ctl->cancel.v, (uint64_t)wall_clock64() + a.timeout_ticks,
                a.cap_wait_ticks, nullptr, kPQ);
      run_query(c);
      flush_counters(c);
      if (l == 0) {
        const uint64_t before = __hip_atomic_fetch_or(&a.join[s], kSlotClosed, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
        // the closing wave also records how many waves are on the query
        const uint32_t on = min(slot_joined(before), slot_want(before));
        const uint32_t add = (before & kSlotClosed) ? 1u : ((on << 16) | 1u);
        const uint32_t fin = __hip_atomic_fetch_add(&c.q.ctrl->finished.v, add, __ATOMIC_ACQ_REL,
                                                    __HIP_MEMORY_SCOPE_AGENT) + add;
        if ((fin >> 16) != 0u && (fin & 0xFFFFu) == (fin >> 16)) {
          // last wave out: every other wave's updates happened before its
          // finished increment; publish status and generation to the host
          const uint32_t err = ld32(&c.q.ctrl->error.v);
          const uint32_t ovf = ld32(&c.q.ctrl->overflow.v);
          const uint64_t word = ((uint64_t)(err | (ovf << 8)) << 32) | slot_gen(before);
          __hip_atomic_store(&a.done_host[s], word, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
      }
      last_busy = (uint64_t)wall_clock64();
      if (l == 0) st32(&a.ctl->last_busy.v, (uint32_t)last_busy);
      idle = 0;
      continue;
    }
    if (uni(ld32(&a.ctl->stop.v))) break;
    // failsafe exit, measured from the last query activity of any wave so that
    // the waves leave together (the host stops an idle server much earlier)
    const uint32_t now = (uint32_t)wall_clock64();
    const uint32_t since = min(now - (uint32_t)last_busy, now - uni(ld32(&a.ctl->last_busy.v)));
    if (since > a.idle_exit_ticks) break;
    ++idle;
    backoff(min(idle >> 2, 6u));
    // long-idle waves poll the slot table less often (up to ~50 us apart)
    for (uint32_t k = idle >> 6; k > 0 && k < 16; --k) __builtin_amdgcn_s_sleep(127);
    if (idle >= 1024) {
      for (uint32_t k = 0; k < 15; ++k) __builtin_amdgcn_s_sleep(127);
    }
  }
}

__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) mlmq_server_worker(ServerArgs a) {
  server_body<false>(a);
}
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) mlmq_server_worker_pq(ServerArgs a) {
  server_body<true>(a);
}

// Per-query reset: dist = UINT32_MAX except dist[source] = 0, all L2 slots
// free except ring 0 / slot 0, which holds the source (it is written through
// to L2 before the worker starts, Section 4.1), counters zero, reservation 1.
// With priority queues every node is empty and unlocked, every heap has no
// node, and queue 0's partial buffer holds the source (pq_in = 1).
__device__ __forceinline__ void init_query(const QueryDesc& q, uint32_t tid, uint32_t stride) {
  const uint32_t n = q.n, src = q.source;
  const bool pq = q.l2_type == MLMQ_L2_PQ;
  uint32_t* dist = q.dist;
  for (uint32_t i = tid; i < n; i += stride) dist[i] = i == src ? 0u : kInf;
  const uint32_t nh = q.nrings << q.nb_log2;
  uint64_t* hdr = q.hdr;
  const uint64_t first = pq ? (1ull << 32) : ((1ull << 32) | 1ull);
  for (uint32_t i = tid; i < nh; i += stride) hdr[i] = i == 0 ? first : 0ull;
  const uint32_t hc = q.hub_cap;
  for (uint32_t i = tid; i < hc; i += stride) {
    q.hub_cur[i] = 0;
    q.hub_pub[i] = 0;
  }
  for (uint32_t i = tid; i < q.nrings; i += stride) {
    q.rings[i].tail.v = (i == 0 && !pq) ? 1u : 0u;
    q.rings[i].head.v = 0;
  }
  const uint32_t cw = sizeof(QueryCtrl) / 4;
  uint32_t* cwp = reinterpret_cast<uint32_t*>(q.ctrl);
  const uint32_t* pq_in = &q.ctrl->pq_in.v;
  for (uint32_t i = tid; i < cw; i += stride) cwp[i] = (pq && cwp + i == pq_in) ? 1u : 0u;
  if (tid == 0) q.data[0] = make_elem(src, 0);
}

__global__ void mlmq_init(const QueryDesc* qs, BatchCtrl* batch) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.y == 0 && tid == 0) {
    batch->cursor.v = 0;
    batch->cancel.v = 0;
  }
  init_query(qs[blockIdx.y], tid, gridDim.x * blockDim.x);
}

// Server admission, step 1: the query's memory is reset as above and its
// descriptor is stored into its slot.
__global__ void mlmq_server_init(QueryDesc q, QueryDesc* slot) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid == 0) *slot = q;
  init_query(q, tid, gridDim.x * blockDim.x);
}

// Server admission, step 2 (a later kernel in the same stream, so every store
// of step 1 is complete): opens the slot.
__global__ void mlmq_server_publish(uint64_t* join, uint64_t word) {
  if (blockIdx.x == 0 && threadIdx.x == 0) __hip_atomic_store(join, word, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Stores one control word (stop / cancel) coherently while the resident
// kernel runs.
__global__ void mlmq_server_signal(uint32_t* p, uint32_t v) {
  if (blockIdx.x == 0 && threadIdx.x == 0) __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Overflow test (exact): some reachable vertex has a distance >= 2^32 - 1 iff
// an edge leaves a finite label towards an unreachable one.
__global__ void mlmq_overflow_check(const QueryDesc* qs, uint32_t* flag) {
  const QueryDesc& q = qs[0];
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < q.n; u += stride) {
    if (q.dist[u] == kInf) continue;
    for (int32_t e = q.off[u]; e < q.off[u + 1]; ++e)
      if (q.dist[(uint32_t)q.adj[e]] == kInf) {
        *flag = 1u;
        break;
      }
  }
}

// Copy every query's status word, overflow flag and counters into one array.
__global__ void mlmq_gather(const QueryDesc* qs, int nq, QueryResult* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  const QueryCtrl* ctl = qs[i].ctrl;
  out[i].error = ctl->error.v;
  out[i].overflow = ctl->overflow.v;
  for (int k = 0; k < kNumCounters; ++k) out[i].stats[k] = ctl->stats[k];
}

// Labels of a solve on the degree-ordered copy of a graph, back in the
// caller's vertex order: out[v] = lab[ord_of[v]].
__global__ void __launch_bounds__(256) mlmq_unorder(const uint32_t* lab, const uint32_t* ord_of, uint32_t n,
                                                    uint32_t* out) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) out[v] = lab[ord_of[v]];
}

// ------------------------------------------------------------ optimality check

// Edges one wave checks per slice; slices are handed out grid-stride.
constexpr uint32_t kCheckSlice = 4096;

// Largest row q in [lo, n) with off[q] <= y, given off[lo] <= y < off[n]: a
// 65-way search in which every lane probes one point per round.
__device__ __forceinline__ uint32_t row_of(const int32_t* off, uint32_t n, uint32_t lo, uint32_t y) {
  uint32_t hi = n;
  while (hi - lo > 1u) {
    const uint32_t span = hi - lo;
    const uint32_t p = lo + (uint32_t)(((uint64_t)span * (lane() + 1u)) / 65u);  // lo <= p < hi
    const bool le = (uint32_t)off[p] <= y;
    const uint64_t ml = ballot(p > lo && le);
    const uint64_t mg = ballot(p > lo && !le);
    if (ml) lo = lane_val(p, 63u - (uint32_t)__clzll((long long)ml));
    if (mg) hi = lane_val(p, first_lane(mg));
  }
  return lo;
}

// Edge pass of the check: for every edge (u, v, w) with dist[u] finite,
// dist[v] must be finite and at most dist[u] + w; an edge with equality marks
// v as having a tight in-edge. The lanes of a wave take 64 consecutive edges;
// their rows come from a window holding the ends of 64 consecutive rows,
// searched by shuffles and moved forward by row_of when an edge lies past it.
__global__ void __launch_bounds__(64) mlmq_check_edges(const int32_t* off, const uint64_t* adj, const uint32_t* dist,
                                                       uint32_t n, uint32_t m, uint8_t* tight,
                                                       unsigned long long* bad) {
  const uint32_t nslices = (m + kCheckSlice - 1u) / kCheckSlice;
  uint32_t nbad = 0;
  for (uint32_t sl = blockIdx.x; sl < nslices; sl += gridDim.x) {
    const uint32_t s = sl * kCheckSlice;
    const uint32_t t = min(m, s + kCheckSlice);
    uint32_t r = row_of(off, n, 0u, s);
    uint32_t endk = (uint32_t)off[min(r + lane() + 1u, n)];  // end of row r + lane
    for (uint32_t x = s; x < t; x += 64u) {
      const uint32_t e = x + lane();
      bool todo = e < t;
      while (ballot(todo)) {
        // rows of the window that end at or before e; exact while e < end of row r + 63
        uint32_t j = 0;
#pragma unroll
        for (uint32_t st = 32; st; st >>= 1)
          if ((uint32_t)__shfl(endk, (int)(j + st - 1u)) <= e) j += st;
        const uint32_t wend = lane_val(endk, 63u);  // end of the window's last row
        const bool in = todo && e < wend;
        if (in) {
          const uint32_t du = dist[r + j];
          if (du != kInf) {
            const uint64_t a = adj[e];
            const uint32_t dv = dist[(uint32_t)a];
            const uint64_t sum = (uint64_t)du + (a >> 32);
            if (dv == kInf || (uint64_t)dv > sum)
              ++nbad;
            else if ((uint64_t)dv == sum)
              tight[(uint32_t)a] = 1;
          }
          todo = false;
        }
        const uint64_t left = ballot(todo);
        if (left) {
          r = row_of(off, n, r, lane_val(e, first_lane(left)));
          endk = (uint32_t)off[min(r + lane() + 1u, n)];
        }
      }
    }
  }
  nbad = wave_sum(nbad);
  if (lane() == 0 && nbad) atomicAdd(bad, (unsigned long long)nbad);
}

// Vertex pass: dist[source] must be 0, and every other vertex with a finite
// distance needs a tight in-edge.
__global__ void __launch_bounds__(256) mlmq_check_vertices(const uint32_t* dist, const uint8_t* tight, uint32_t n,
                                                           uint32_t source, unsigned long long* bad) {
  uint32_t nbad = 0;
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const uint32_t d = dist[v];
    if (v == source)
      nbad += d != 0u;
    else
      nbad += (d != kInf && tight[v] == 0);
  }
  nbad = wave_sum(nbad);
  if (lane() == 0 && nbad) atomicAdd(bad, (unsigned long long)nbad);
}

// ------------------------------------------------------------ latency probes

// Dependent-hop chain: lane 0 of one wave walks `hops` hops from v0; each hop
// loads the row bounds of the current vertex, then one of its edge words
// (picked by the hop number), then takes an agent-scope atomicMin on the
// neighbour's label, and the next vertex depends on the value the atomic
// returned -- the three memory operations of one relaxation, each waiting for
// the one before, with no queue in between. out[0] = wall-clock ticks.
__global__ void __launch_bounds__(64) mlmq_hop_probe(const int32_t* off, const uint64_t* adj, uint32_t* lab,
                                                    uint32_t n, uint32_t v0, uint32_t hops, uint64_t* out) {
  if (threadIdx.x != 0) return;
  uint32_t v = v0;
  const uint64_t t0 = (uint64_t)wall_clock64();
  for (uint32_t i = 0; i < hops; ++i) {
    const int32_t b = off[v], e = off[v + 1];
    if (e <= b) {
      v = v0;
      continue;
    }
    const uint64_t a = adj[(uint32_t)b + i % (uint32_t)(e - b)];
    const uint32_t u = (uint32_t)a;
    const uint32_t old = __hip_atomic_fetch_min(lab + u, i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    v = u + (old == 0xFFFFFFFEu ? 1u : 0u);  // never taken, but waits for the atomic
    if (v >= n) v = v0;
  }
  out[0] = (uint64_t)wall_clock64() - t0;
}

// Hand-off between two workgroups (placed on different XCDs by the round-robin
// dispatch): they take turns incrementing one agent-scope word, each waiting
// to see the other's value -- the round trip of publishing work that another
// wave picks up. Every wait gives up at the deadline (out[1] = 1 then).
// out[0] = ticks for `rounds` round trips, measured by workgroup 0.
__global__ void __launch_bounds__(64) mlmq_handoff_probe(uint32_t* word, uint32_t rounds, uint64_t limit_ticks,
                                                        uint64_t* out) {
  if (threadIdx.x != 0 || blockIdx.x > 1) return;
  const uint32_t me = blockIdx.x;
  const uint64_t t0 = (uint64_t)wall_clock64();
  for (uint32_t r = 0; r < rounds; ++r) {
    const uint32_t want = 2u * r + me;  // workgroup 0 moves on even values, 1 on odd ones
    while (__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != want) {
      if ((uint64_t)wall_clock64() - t0 > limit_ticks) {
        if (me == 0) out[1] = 1;
        return;
      }
    }
    __hip_atomic_store(word, want + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (me == 0) out[0] = (uint64_t)wall_clock64() - t0;
}

// ------------------------------------------------------------ host launchers

size_t worker_lds_bytes(uint32_t waves, uint32_t l1_cap, bool two_rings, bool stage) {
  (void)waves;
  return 8ull * (64ull + (uint64_t)l1_cap * (two_rings ? 2u : 1u) + (stage ? 64ull * kStageB : 0ull));
}

hipError_t launch_init(const QueryDesc* d_queries, BatchCtrl* d_batch, int nq, uint32_t max_words, hipStream_t s) {
  uint32_t blocks = (max_words + 255u) / 256u;
  blocks = blocks < 1u ? 1u : (blocks > 2048u ? 2048u : blocks);
  hipLaunchKernelGGL(mlmq_init, dim3(blocks, (uint32_t)nq), dim3(256), 0, s, d_queries, d_batch);
  return hipGetLastError();
}

hipError_t launch_worker(const LaunchArgs& a, uint32_t grid, uint32_t wg_size, size_t lds, hipStream_t s) {
  if (a.pq)
    hipLaunchKernelGGL(mlmq_worker_pq, dim3(grid), dim3(wg_size), lds, s, a);
  else
    hipLaunchKernelGGL(mlmq_worker, dim3(grid), dim3(wg_size), lds, s, a);
  return hipGetLastError();
}

// The admission-side kernels below run in one-wave workgroups, so that they
// fit into any free wave slot beside a resident server kernel.
hipError_t launch_overflow_check(const QueryDesc* d_query, uint32_t* d_flag, hipStream_t s) {
  hipLaunchKernelGGL(mlmq_overflow_check, dim3(4096), dim3(64), 0, s, d_query, d_flag);
  return hipGetLastError();
}

hipError_t launch_unorder(const uint32_t* d_lab, const uint32_t* d_ord_of, uint32_t n, uint32_t* d_out, hipStream_t s) {
  uint32_t blocks = (n + 255u) / 256u;
  blocks = blocks < 1u ? 1u : (blocks > 16384u ? 16384u : blocks);
  hipLaunchKernelGGL(mlmq_unorder, dim3(blocks), dim3(256), 0, s, d_lab, d_ord_of, n, d_out);
  return hipGetLastError();
}

hipError_t launch_gather(const QueryDesc* d_queries, int nq, QueryResult* d_out, hipStream_t s) {
  hipLaunchKernelGGL(mlmq_gather, dim3((uint32_t)(nq + 255) / 256u), dim3(256), 0, s, d_queries, nq, d_out);
  return hipGetLastError();
}

hipError_t launch_server_worker(const ServerArgs& a, uint32_t grid, size_t lds, hipStream_t s) {
  if (a.pq)
    hipLaunchKernelGGL(mlmq_server_worker_pq, dim3(grid), dim3(64), lds, s, a);
  else
    hipLaunchKernelGGL(mlmq_server_worker, dim3(grid), dim3(64), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_server_admit(const QueryDesc& q, QueryDesc* d_slot, uint64_t* d_join, uint64_t word,
                               uint32_t max_words, hipStream_t s) {
  uint32_t blocks = (max_words + 63u) / 64u;
  blocks = blocks < 1u ? 1u : (blocks > 8192u ? 8192u : blocks);
  hipLaunchKernelGGL(mlmq_server_init, dim3(blocks), dim3(64), 0, s, q, d_slot);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlmq_server_publish, dim3(1), dim3(64), 0, s, d_join, word);
  return hipGetLastError();
}

hipError_t launch_server_signal(uint32_t* d_word, uint32_t v, hipStream_t s) {
  hipLaunchKernelGGL(mlmq_server_signal, dim3(1), dim3(64), 0, s, d_word, v);
  return hipGetLastError();
}

hipError_t launch_check(const int32_t* off, const uint64_t* adj, const uint32_t* dist, uint32_t n, uint32_t m,
                        uint32_t source, uint8_t* tight, unsigned long long* bad, hipEvent_t ev0, hipEvent_t ev1,
                        hipStream_t s) {
  const uint32_t nslices = (m + kCheckSlice - 1u) / kCheckSlice;
  const uint32_t grid = nslices < 1u ? 1u : (nslices > 8192u ? 8192u : nslices);
  hipError_t e = hipEventRecord(ev0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlmq_check_edges, dim3(grid), dim3(64), 0, s, off, adj, dist, n, m, tight, bad);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipEventRecord(ev1, s);
  if (e != hipSuccess) return e;
  uint32_t vb = (n + 255u) / 256u;
  vb = vb < 1u ? 1u : (vb > 4096u ? 4096u : vb);
  hipLaunchKernelGGL(mlmq_check_vertices, dim3(vb), dim3(256), 0, s, dist, tight, n, source, bad);
  return hipGetLastError();
}

hipError_t launch_latency_probes(const int32_t* off, const uint64_t* adj, uint32_t* lab, uint32_t n, uint32_t v0,
                                 uint32_t hops, uint32_t* word, uint32_t rounds, uint64_t limit_ticks, uint64_t* out,
                                 hipStream_t s) {
  hipLaunchKernelGGL(mlmq_hop_probe, dim3(1), dim3(64), 0, s, off, adj, lab, n, v0, hops, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlmq_handoff_probe, dim3(2), dim3(64), 0, s, word, rounds, limit_ticks, out + 2);
  return hipGetLastError();
}

hipError_t server_occupancy(size_t lds, bool pq, int* wgs_per_cu) {
  return pq ? hipOccupancyMaxActiveBlocksPerMultiprocessor(wgs_per_cu, mlmq_server_worker_pq, 64, lds)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(wgs_per_cu, mlmq_server_worker, 64, lds);
}

hipError_t worker_occupancy(uint32_t wg_size, size_t lds, bool pq, int* wgs_per_cu) {
  return pq ? hipOccupancyMaxActiveBlocksPerMultiprocessor(wgs_per_cu, mlmq_worker_pq, (int)wg_size, lds)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(wgs_per_cu, mlmq_worker, (int)wg_size, lds);
}

// ------------------------------------------------------------ allocation-free solve

// Queue memory of the allocation-free single-source solve: one fixed array on
// every device the library runs on, reserved with the code object and held
// until the process ends. On the host the name `scratch` is only a stand-in
// for the device symbol; host code uses the device address below instead,
// taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace mlmq
