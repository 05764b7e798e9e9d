// Runs the library's init and persistent worker kernels on the CPU (one host
// thread per lane) for small graphs. Test infrastructure only.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "sim_kernels.inc"

namespace simt {
thread_local unsigned lane;
thread_local Wave* wave;
thread_local Group* group;
thread_local dim3 tidx, bidx, bdim, gdim;
thread_local uint64_t nops;
bool check_stacks = getenv("SIM_STACKS") != nullptr;
}  // namespace simt

using namespace mlmq;

namespace {
// Device memory and LDS start with whatever was there before; mimic that
// with a fixed garbage pattern unless SIM_ZERO is set.
template <class T>
T* zalloc(size_t count) {
  void* p = nullptr;
  const size_t bytes = sizeof(T) * (count ? count : 1);
  if (posix_memalign(&p, 256, bytes)) abort();
  if (getenv("SIM_ZERO")) {
    std::memset(p, 0, bytes);
  } else {
    uint64_t x = 0x9E3779B97F4A7C15ull ^ bytes;
    uint8_t* b = static_cast<uint8_t*>(p);
    for (size_t i = 0; i < bytes; ++i) {
      x ^= x << 13;
      x ^= x >> 7;
      x ^= x << 17;
      b[i] = (uint8_t)x;
    }
  }
  return static_cast<T*>(p);
}
}  // namespace

// knobs: l0_rows, l1_type, l2_type, l1_cap, l1_wb, delta1, d2_log2, bmax, bnum,
//        th_v, th_hub, hub_chunk, nb_log2, hub_cap, timeout_ms, relax_mode, unit_w
extern "C" int sim_sssp(int32_t n, const int32_t* off, const int32_t* col, const uint32_t* w, uint32_t src,
                        uint32_t* dist, const uint32_t* k, uint32_t nwg, uint32_t wg_size, uint64_t* stats,
                        uint32_t* status) {
  const int64_t m = off[n];
  std::vector<uint64_t> adj((size_t)m + 1);
  for (int64_t e = 0; e < m; ++e) adj[e] = (uint32_t)col[e] | ((uint64_t)w[e] << 32);
  const uint32_t nrings = k[2] == 1 ? k[7] : (k[2] == 2 ? k[17] : 1);
  const uint32_t nb_log2 = k[12], hub_cap = k[13];
  const uint64_t nh = (uint64_t)nrings << nb_log2;
  QueryCtrl* ctrl = zalloc<QueryCtrl>(1);
  RingCtr* rings = zalloc<RingCtr>(nrings);
  uint64_t* hdr = zalloc<uint64_t>(nh);
  uint64_t* data = zalloc<uint64_t>(nh * 64);
  uint64_t* hub_rec = zalloc<uint64_t>(2ull * hub_cap);
  uint32_t* hub_cur = zalloc<uint32_t>(hub_cap);
  uint32_t* hub_pub = zalloc<uint32_t>(hub_cap);
  BatchCtrl* batch = zalloc<BatchCtrl>(1);
  QueryDesc* q = zalloc<QueryDesc>(1);
  q->off = off;
  q->adj = adj.data();
  q->dist = dist;
  q->ctrl = ctrl;
  q->rings = rings;
  q->hdr = hdr;
  q->data = data;
  q->hub_rec = hub_rec;
  q->hub_cur = hub_cur;
  q->hub_pub = hub_pub;
  q->n = (uint32_t)n;
  q->source = src;
  q->nb_log2 = nb_log2;
  q->nrings = nrings;
  q->hub_cap = hub_cap;
  q->l0_cap = 64u * k[0];
  q->l1_type = k[1];
  q->l2_type = k[2];
  q->l1_cap = k[1] == MLMQ_L1_NONE ? 64u : k[3];
  q->l1_wb = k[4];
  q->delta1 = k[5];
  q->d2_log2 = k[6];
  q->bnum = k[2] == 1 ? k[8] : 1;
  q->th_v = k[9];
  q->th_hub = k[10];
  q->hub_chunk = k[11];
  q->want_wgs = nwg;
  q->relax_mode = k[15];
  q->unit_w = k[16];
  q->donate_min = 32;
  // init kernel, serially over its threads (it has no cross-lane operations)
  const uint32_t blocks = 4;
  simt::gdim = dim3(blocks, 1);
  simt::bdim = dim3(256);
  for (uint32_t b = 0; b < blocks; ++b)
    for (uint32_t t = 0; t < 256; ++t) {
      simt::bidx = dim3(b, 0);
      simt::tidx = dim3(t);
      mlmq_init(q, batch);
    }
  // persistent worker: nwg workgroups x wg_size lane threads
  const uint32_t waves = wg_size / 64;
  const uint32_t l1cap = q->l1_cap;
  const bool two = k[1] == MLMQ_L1_NEARFAR;
  const bool stage = k[2] == 1;
  const size_t lds = worker_lds_bytes(waves, l1cap, two, stage);
  LaunchArgs a;
  std::memset(&a, 0, sizeof(a));
  a.queries = q;
  a.batch = batch;
  a.nq = 1;
  a.l1_cap = l1cap;
  a.l1_two = two;
  a.stage = stage;
  a.waves = waves;
  a.timeout_ticks = (uint64_t)k[14] * 100000ull;
  a.cap_wait_ticks = 200ull * 100000ull;
  std::vector<uint32_t> beats(nwg * waves, 0);
  a.beats = getenv("SIM_DUMP") ? beats.data() : nullptr;
  std::vector<simt::Wave*> wv;
  std::vector<simt::Group> grp(nwg);
  std::vector<std::barrier<>*> bars;
  std::vector<uint8_t*> ldsb;
  for (uint32_t g = 0; g < nwg; ++g) {
    bars.push_back(new std::barrier<>(wg_size));
    ldsb.push_back(zalloc<uint8_t>(lds));
    grp[g].bar = bars.back();
    grp[g].lds = ldsb.back();
    for (uint32_t w2 = 0; w2 < waves; ++w2) wv.push_back(new simt::Wave());
  }
  std::vector<std::thread> th;
  for (uint32_t g = 0; g < nwg; ++g)
    for (uint32_t t = 0; t < wg_size; ++t)
      th.emplace_back([&, g, t] {
        simt::lane = t % 64;
        simt::nops = 0;
        simt::wave = wv[g * waves + t / 64];
        simt::group = &grp[g];
        simt::tidx = dim3(t);
        simt::bidx = dim3(g);
        simt::bdim = dim3(wg_size);
        simt::gdim = dim3(nwg);
        if (k[2] == MLMQ_L2_PQ)
          mlmq_worker_pq(a);
        else
          mlmq_worker(a);
      });
  for (auto& t : th) t.join();
  if (getenv("SIM_DUMP")) {
    fprintf(stderr, "done %u term %u err %u cur %u hub_units %u\n", ctrl->done.v, ctrl->terminate.v, ctrl->error.v,
            ctrl->cur.v, ctrl->hub_units.v);
    for (uint32_t r = 0; r < nrings; ++r)
      if (rings[r].tail.v || rings[r].head.v) fprintf(stderr, "  ring %u tail %u head %u\n", r, rings[r].tail.v, rings[r].head.v);
    for (uint32_t i = 0; i < nwg * waves; ++i) fprintf(stderr, "  wave %u point %u it %u\n", i, beats[i] >> 24, beats[i] & 0xFFFFFF);
  }
  for (int i = 0; i < kNumCounters && stats; ++i) stats[i] = ctrl->stats[i];
  if (status) {
    status[0] = ctrl->error.v;
    status[1] = ctrl->overflow.v;
    status[2] = ctrl->done.v;
    status[3] = rings[0].tail.v;
  }
  for (auto* p : wv) delete p;
  for (auto* p : bars) delete p;
  for (auto* p : ldsb) free(p);
  free(ctrl);
  free(rings);
  free(hdr);
  free(data);
  free(hub_rec);
  free(hub_cur);
  free(hub_pub);
  free(batch);
  free(q);
  return 0;
}

// Runs f on every lane thread of nwg workgroups of `block` lanes.
template <class F>
static void run_grid(uint32_t nwg, uint32_t block, F f) {
  const uint32_t waves = block / 64;
  std::vector<simt::Wave*> wv;
  std::vector<simt::Group> grp(nwg);
  std::vector<std::barrier<>*> bars;
  for (uint32_t g = 0; g < nwg; ++g) {
    bars.push_back(new std::barrier<>(block));
    grp[g].bar = bars.back();
    grp[g].lds = nullptr;
    for (uint32_t w2 = 0; w2 < waves; ++w2) wv.push_back(new simt::Wave());
  }
  std::vector<std::thread> th;
  for (uint32_t g = 0; g < nwg; ++g)
    for (uint32_t t = 0; t < block; ++t)
      th.emplace_back([&, g, t] {
        simt::lane = t % 64;
        simt::nops = 0;
        simt::wave = wv[g * waves + t / 64];
        simt::group = &grp[g];
        simt::tidx = dim3(t);
        simt::bidx = dim3(g);
        simt::bdim = dim3(block);
        simt::gdim = dim3(nwg);
        f();
      });
  for (auto& t : th) t.join();
  for (auto* p : wv) delete p;
  for (auto* p : bars) delete p;
}

// The queue-unit example: distances 5, 1, 2 written to one wave's L1 one at a
// time (vertices 0, 1, 2), then one L1 read. read_d receives the distances
// read, in lane order (*nread of them); left_d what stays in L1 (near ring,
// then far ring); l2_d what went to the global level (ring 0, block 0).
extern "C" int sim_l1_example(uint32_t l1_type, uint32_t delta1, uint32_t* read_d, uint32_t* nread, uint32_t* left_d,
                              uint32_t* nleft, uint32_t* l2_d, uint32_t* nl2) {
  const uint32_t nb_log2 = 4, cap = 64;
  QueryCtrl* ctrl = zalloc<QueryCtrl>(1);
  RingCtr* rings = zalloc<RingCtr>(1);
  uint64_t* hdr = zalloc<uint64_t>(1u << nb_log2);
  uint64_t* data = zalloc<uint64_t>((1u << nb_log2) * 64);
  uint32_t dist[3] = {kInf, kInf, kInf};
  // what the init kernel would leave: empty counters, every L2 slot free for lap 0
  std::memset(ctrl, 0, sizeof(QueryCtrl));
  std::memset(rings, 0, sizeof(RingCtr));
  std::memset(hdr, 0, sizeof(uint64_t) << nb_log2);
  QueryDesc* q = zalloc<QueryDesc>(1);
  std::memset(q, 0, sizeof(QueryDesc));
  q->dist = dist;
  q->ctrl = ctrl;
  q->rings = rings;
  q->hdr = hdr;
  q->data = data;
  q->n = 3;
  q->nb_log2 = nb_log2;
  q->nrings = 1;
  q->hub_cap = 1;
  q->l1_type = l1_type;
  q->l2_type = MLMQ_L2_FIFO;
  q->l1_cap = cap;
  q->delta1 = delta1;
  q->bnum = 1;
  q->th_v = 32;
  q->want_wgs = 1;
  const bool two = l1_type == MLMQ_L1_NEARFAR;
  uint8_t* lds = zalloc<uint8_t>(worker_lds_bytes(1, cap, two, false));
  uint32_t cancel = 0;
  run_grid(1, 64, [&] {
    simt::group->lds = lds;
    Ctx c;
    setup_ctx(c, *q, reinterpret_cast<uint64_t*>(lds), cap, two ? 1u : 0u, 0u, &cancel, ~0ull >> 1, 1000000ull,
              nullptr, false);
    const uint32_t ds[3] = {5, 1, 2};
    for (uint32_t i = 0; i < 3; ++i) write_l1(c, make_elem(i, ds[i]), lane() == 0);
    uint64_t e = 0;
    bool ok = false;
    l1_take(c, e, ok);
    const uint32_t k = popc(ballot(ok));
    if (ok) read_d[lane()] = elem_d(e);
    if (lane() == 0) {
      *nread = k;
      uint32_t j = 0;
      for (uint32_t x = c.qh; x != c.qt; ++x) left_d[j++] = elem_d(c.l1[x & c.l1mask]);
      for (uint32_t x = c.fh; x != c.ft; ++x) left_d[j++] = elem_d(c.far[x & c.l1mask]);
      *nleft = j;
    }
  });
  // a written L2 block: its header holds the element count, data the elements
  uint32_t j = 0;
  if (rings[0].tail.v) {
    const uint32_t cnt = (uint32_t)hdr[0];  // low half: element count; high half: lap state
    for (uint32_t x = 0; x < cnt && x < 64; ++x) l2_d[j++] = (uint32_t)(data[x] >> 32);
  }
  *nl2 = j;
  free(ctrl);
  free(rings);
  free(hdr);
  free(data);
  free(q);
  free(lds);
  return 0;
}

// Optimality check: edge pass on nwg one-wave workgroups, then the vertex
// pass on one 256-lane workgroup; *bad_out receives the violation count.
extern "C" int sim_check(int32_t n, const int32_t* off, const int32_t* col, const uint32_t* w, uint32_t src,
                         const uint32_t* dist, uint32_t nwg, uint64_t* bad_out) {
  const uint32_t m = (uint32_t)off[n];
  std::vector<uint64_t> adj((size_t)m + 1);
  for (uint32_t e = 0; e < m; ++e) adj[e] = (uint32_t)col[e] | ((uint64_t)w[e] << 32);
  std::vector<uint8_t> tight((size_t)n, 0);
  unsigned long long bad = 0;
  run_grid(nwg, 64, [&] { mlmq_check_edges(off, adj.data(), dist, (uint32_t)n, m, tight.data(), &bad); });
  run_grid(1, 256, [&] { mlmq_check_vertices(dist, tight.data(), (uint32_t)n, src, &bad); });
  *bad_out = bad;
  return 0;
}

// Serving form: nq queries (sources srcs[i], outputs dist + i * n) through the
// resident server kernel with nslots slots and nwg one-wave workgroups. A host
// driver thread plays the library's admission loop: it resets a query's memory
// (init kernel, run serially), opens its slot (publish kernel), watches the
// completion words, and admits the next query in arrival order.
extern "C" int sim_server(int32_t n, const int32_t* off, const int32_t* col, const uint32_t* w, int32_t nq,
                          const uint32_t* srcs, uint32_t* dist, const uint32_t* k, uint32_t nwg, int32_t nslots,
                          uint32_t want, uint32_t* status) {
  const int64_t m = off[n];
  std::vector<uint64_t> adj((size_t)m + 1);
  for (int64_t e = 0; e < m; ++e) adj[e] = (uint32_t)col[e] | ((uint64_t)w[e] << 32);
  const uint32_t nrings = k[2] == 1 ? k[7] : (k[2] == 2 ? k[17] : 1);
  const uint32_t nb_log2 = k[12], hub_cap = k[13];
  const uint64_t nh = (uint64_t)nrings << nb_log2;
  QueryDesc* slots = zalloc<QueryDesc>(64);
  uint64_t* join = zalloc<uint64_t>(64);
  uint64_t* done = zalloc<uint64_t>(64);
  ServerCtrl* ctl = zalloc<ServerCtrl>(1);
  for (int i = 0; i < 64; ++i) {
    join[i] = 1ull << 31;  // closed
    done[i] = 0;
  }
  ctl->stop.v = 0;
  ctl->cancel.v = 0;
  const uint32_t l1cap = k[1] == MLMQ_L1_NONE ? 64u : k[3];
  const bool two = k[1] == MLMQ_L1_NEARFAR;
  const bool stage = k[2] == 1;
  const size_t lds = worker_lds_bytes(1, l1cap, two, stage);
  ServerArgs a;
  std::memset(&a, 0, sizeof(a));
  a.slots = slots;
  a.join = join;
  a.done_host = done;
  a.ctl = ctl;
  a.nslots = nslots;
  a.l1_cap = l1cap;
  a.l1_two = two;
  a.stage = stage;
  a.timeout_ticks = (uint64_t)k[14] * 100000ull;
  a.cap_wait_ticks = 200ull * 100000ull;
  a.idle_exit_ticks = (uint64_t)k[14] * 100000ull;

  std::vector<simt::Wave*> wv;
  std::vector<simt::Group> grp(nwg);
  std::vector<std::barrier<>*> bars;
  std::vector<uint8_t*> ldsb;
  for (uint32_t g = 0; g < nwg; ++g) {
    bars.push_back(new std::barrier<>(64));
    ldsb.push_back(zalloc<uint8_t>(lds));
    grp[g].bar = bars.back();
    grp[g].lds = ldsb.back();
    wv.push_back(new simt::Wave());
  }
  std::vector<std::thread> th;
  for (uint32_t g = 0; g < nwg; ++g)
    for (uint32_t t = 0; t < 64; ++t)
      th.emplace_back([&, g, t] {
        simt::lane = t;
        simt::nops = 0;
        simt::wave = wv[g];
        simt::group = &grp[g];
        simt::tidx = dim3(t);
        simt::bidx = dim3(g);
        simt::bdim = dim3(64);
        simt::gdim = dim3(nwg);
        if (k[2] == MLMQ_L2_PQ)
          mlmq_server_worker_pq(a);
        else
          mlmq_server_worker(a);
      });

  struct Mem {
    QueryCtrl* ctrl;
    RingCtr* rings;
    uint64_t *hdr, *data, *hub_rec;
    uint32_t *hub_cur, *hub_pub;
  };
  std::vector<int32_t> slot_q(nslots, -1);
  std::vector<uint32_t> slot_gen(nslots, 0);
  std::vector<Mem> slot_mem(nslots);
  int32_t next = 0, finished = 0;
  uint32_t gen = 1;
  const auto t_end = std::chrono::steady_clock::now() + std::chrono::milliseconds(k[14] + 5000);
  while (finished < nq && std::chrono::steady_clock::now() < t_end) {
    for (int32_t s = 0; s < nslots; ++s) {
      if (slot_q[s] >= 0) {
        const uint64_t wd = __atomic_load_n(&done[s], __ATOMIC_ACQUIRE);
        if ((uint32_t)wd != slot_gen[s]) continue;
        status[slot_q[s]] = (uint32_t)(wd >> 32);
        Mem& mm = slot_mem[s];
        free(mm.ctrl), free(mm.rings), free(mm.hdr), free(mm.data), free(mm.hub_rec), free(mm.hub_cur),
            free(mm.hub_pub);
        slot_q[s] = -1;
        ++finished;
      }
      if (slot_q[s] < 0 && next < nq) {
        const int32_t qi = next++;
        Mem mm{zalloc<QueryCtrl>(1), zalloc<RingCtr>(nrings), zalloc<uint64_t>(nh), zalloc<uint64_t>(nh * 64),
               zalloc<uint64_t>(2ull * hub_cap), zalloc<uint32_t>(hub_cap), zalloc<uint32_t>(hub_cap)};
        QueryDesc q;
        std::memset(&q, 0, sizeof(q));
        q.off = off;
        q.adj = adj.data();
        q.dist = dist + (size_t)qi * n;
        q.ctrl = mm.ctrl;
        q.rings = mm.rings;
        q.hdr = mm.hdr;
        q.data = mm.data;
        q.hub_rec = mm.hub_rec;
        q.hub_cur = mm.hub_cur;
        q.hub_pub = mm.hub_pub;
        q.n = (uint32_t)n;
        q.source = srcs[qi];
        q.nb_log2 = nb_log2;
        q.nrings = nrings;
        q.hub_cap = hub_cap;
        q.l0_cap = 64u * k[0];
        q.l1_type = k[1];
        q.l2_type = k[2];
        q.l1_cap = l1cap;
        q.l1_wb = k[4];
        q.delta1 = k[5];
        q.d2_log2 = k[6];
        q.bnum = k[2] == 1 ? k[8] : 1;
        q.th_v = k[9];
        q.th_hub = k[10];
        q.hub_chunk = k[11];
        q.want_wgs = want;
        q.relax_mode = k[15];
        q.unit_w = k[16];
        q.donate_min = 32;
        __atomic_store_n(&done[s], 0ull, __ATOMIC_RELEASE);
        simt::gdim = dim3(4, 1);
        simt::bdim = dim3(256);
        for (uint32_t b = 0; b < 4; ++b)
          for (uint32_t t = 0; t < 256; ++t) {
            simt::bidx = dim3(b, 0);
            simt::tidx = dim3(t);
            mlmq_server_init(q, slots + s);
          }
        simt::gdim = dim3(1);
        simt::bdim = dim3(64);
        simt::bidx = dim3(0);
        simt::tidx = dim3(0);
        mlmq_server_publish(join + s, ((uint64_t)gen << 32) | ((uint64_t)want << 16));
        slot_q[s] = qi;
        slot_gen[s] = gen++;
        slot_mem[s] = mm;
      }
    }
    std::this_thread::yield();
  }
  __atomic_store_n(&ctl->stop.v, 1u, __ATOMIC_SEQ_CST);
  for (auto& t : th) t.join();
  for (auto* p : wv) delete p;
  for (auto* p : bars) delete p;
  for (auto* p : ldsb) free(p);
  free(slots);
  free(join);
  free(done);
  free(ctl);
  return finished == nq ? 0 : -1;
}

// Priority queues alone (Section 4.2, L2PQ / L2MPQ): nwaves one-wave
// workgroups each write `rounds` batches of 1..64 random elements (element
// ids unique: wave << 20 | round << 6 | lane) into pnum queues, taking one
// batch after every `pop_every` writes; afterwards one wave takes everything
// left. Every element written lands in ins[] and every element taken in
// out[] (counts in *nin, *nout); *unsorted counts taken batches that are not
// ascending, and with a single wave and pop_every = 0, *disorder counts
// taken elements smaller than one taken before (an exact priority queue
// gives 0). status: [device status, pq_in, elements still queued].
extern "C" int sim_pq(uint32_t nwaves, uint32_t pnum, uint32_t nb_log2, uint32_t rounds, uint32_t pop_every,
                      uint32_t dmax, uint64_t seed, uint64_t* ins, uint32_t* nin, uint64_t* out, uint32_t* nout,
                      uint32_t* unsorted, uint32_t* disorder, uint32_t* status) {
  const uint64_t nh = (uint64_t)pnum << nb_log2;
  QueryCtrl* ctrl = zalloc<QueryCtrl>(1);
  RingCtr* rings = zalloc<RingCtr>(pnum);
  uint64_t* hdr = zalloc<uint64_t>(nh);
  uint64_t* data = zalloc<uint64_t>(nh * 64);
  // what the init kernel leaves for priority queues with no source element
  std::memset(ctrl, 0, sizeof(QueryCtrl));
  std::memset(rings, 0, sizeof(RingCtr) * pnum);
  std::memset(hdr, 0, sizeof(uint64_t) * nh);
  QueryDesc* q = zalloc<QueryDesc>(1);
  std::memset(q, 0, sizeof(QueryDesc));
  q->ctrl = ctrl;
  q->rings = rings;
  q->hdr = hdr;
  q->data = data;
  q->n = 1u << 30;
  q->nb_log2 = nb_log2;
  q->nrings = pnum;
  q->hub_cap = 1;
  q->l1_type = MLMQ_L1_NONE;
  q->l2_type = MLMQ_L2_PQ;
  q->l1_cap = 64;
  q->bnum = 1;
  q->th_v = 32;
  q->want_wgs = nwaves;
  uint32_t cancel = 0;
  std::atomic<uint32_t> ni{0}, no{0}, bad_batches{0};
  const uint64_t limit = 60ull * 1000 * 100000ull;  // 60 s of wall-clock ticks
  auto take = [&](Ctx& c, uint32_t& last_d, bool track) {
    uint64_t e = 0;
    bool ok = false;
    const bool got = pq_read(c, e, ok);
    if (!got) return false;
    // ascending within the batch: each taken lane is >= the previous lane
    const uint64_t prev = shfl64(e, lane() ? lane() - 1u : 0u);
    const bool okp = __shfl((int)ok, lane() ? (int)lane() - 1 : 0) != 0;
    if (ballot(ok && lane() > 0 && okp && e < prev)) bad_batches++;
    const uint64_t m = ballot(ok);
    uint32_t base = 0;
    if (lane() == 0) base = no.fetch_add(popc(m));
    base = lane_val(base, 0);
    if (ok) out[base + rank_of(m)] = e;
    if (track) {
      // the batch is ascending (checked above): compare its first element
      // with the last one taken before, then remember its last
      const uint32_t k = popc(m);
      const uint32_t first = lane_val(elem_d(e), 0), lastb = lane_val(elem_d(e), k - 1u);
      if (lane() == 0 && first < last_d) (*disorder)++;
      last_d = lastb;
    }
    return true;
  };
  *disorder = 0;
  run_grid(nwaves, 64, [&] {
    Ctx c;
    setup_ctx(c, *q, nullptr, 64, 0u, 0u, &cancel, (uint64_t)wall_clock64() + limit, 1000000ull, nullptr, true);
    uint64_t x = seed ^ (0x9E3779B97F4A7C15ull * (blockIdx.x + 1u));
    uint32_t last_d = 0;
    for (uint32_t r = 0; r < rounds && !c.stop; ++r) {
      x = x * 6364136223846793005ull + 1442695040888963407ull;
      const uint32_t k = 1u + (uint32_t)((x >> 33) % 64u);
      uint64_t y = x ^ (0xD1B54A32D192ED03ull * (lane() + 1u));
      y ^= y >> 29;
      y *= 0xBF58476D1CE4E5B9ull;
      y ^= y >> 32;
      const bool ok = lane() < k;
      const uint64_t e = make_elem((blockIdx.x << 20) | (r << 6) | lane(), (uint32_t)(y % dmax));
      const uint64_t m = ballot(ok);
      uint32_t base = 0;
      if (lane() == 0) base = ni.fetch_add(popc(m));
      base = lane_val(base, 0);
      if (ok) ins[base + rank_of(m)] = e;
      pq_write(c, e, ok);
      if (pop_every && (r % pop_every) == pop_every - 1u) take(c, last_d, false);
    }
    if (c.stop && lane() == 0) status[0] = ctrl->error.v;
  });
  run_grid(1, 64, [&] {
    Ctx c;
    setup_ctx(c, *q, nullptr, 64, 0u, 0u, &cancel, (uint64_t)wall_clock64() + limit, 1000000ull, nullptr, true);
    uint32_t last_d = 0;
    const bool track = nwaves == 1 && pop_every == 0;
    while (!c.stop && take(c, last_d, track)) {
    }
  });
  status[0] = ctrl->error.v;
  status[1] = ctrl->pq_in.v;
  uint32_t left = 0;
  for (uint32_t i = 0; i < pnum; ++i) left += rings[i].tail.v * 64u + (uint32_t)(hdr[(uint64_t)i << nb_log2] >> 32);
  status[2] = left;
  *nin = ni.load();
  *nout = no.load();
  *unsorted = bad_batches.load();
  free(ctrl);
  free(rings);
  free(hdr);
  free(data);
  free(q);
  return 0;
}
