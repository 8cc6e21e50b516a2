// serve.cpp -- batched fixpoints for serving: many independent closure
// (repeated squaring) and same-generation requests, resident in one device
// pool, advanced together by one grouped launch per round.
//
// A request is admitted with dl_batch_submit or dl_batch_submit_edges (its
// relation is normalised into pool buffers, padded to a multiple of 64 for
// n <= 256, of 128 up to 1024, else of 256).  Each dl_batch_step is one round:
// every unfinished request advances by one product -- a closure request by one
// squaring step R' = [A + R R], a same-generation request by one of the two
// products of its step (T = [P S], then S' = [I + T P^T]) -- in up to three
// persistent launches over the concatenated tile lists of the requests of
// each tile size (64 x 64, 128 x 128, and the 256 x 256 direct-to-LDS tiles).
// The round ends
// with one read-back of the per-request model sizes; a request whose model
// size repeats is finished (its iteration count follows the same convention
// as dl_tc/dl_sg) and can be fetched, which frees its slot and pool memory.
// Requests can be submitted between any two rounds, so batching is
// continuous at the granularity of one product.
//
// With one round of look-ahead (dl_batch_set_lookahead), a dl_batch_step
// enqueues the next round before it waits for the one already on the device,
// so the host's bookkeeping between rounds overlaps the device's products.
// The next round is built before the current one's model sizes are known: a
// request that may finish in round k still gets a round k + 1 product, with a
// test the device evaluates once round k is done (its counter against the
// value that means "model size repeated"); k_group_upload then gives that
// product no tiles, so finished requests cost the round nothing (their
// product would write only the buffer that does not hold the model).  Each
// round has its own counter, descriptor and read-back set (two sets
// alternate); a round's entries carry the request's admission number, so a
// slot fetched and reused meanwhile is not confused with its previous
// request; pool memory released by dl_batch_fetch returns to the pool only
// after the round that may still read it has completed.
//
// Per round the device sees one descriptor upload (all tile lists), the
// grouped launches and one counter read-back.  The round counters are never
// cleared: every round of a set reads all of that set's counters back, so a
// product's count is the difference from the value read in the set's
// previous round.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/dl.h"
#include "common.h"

using namespace dl;

namespace dl {
void set_last_error(const std::string& m);
}

namespace {

int bfail(int st, const std::string& m) {
  dl::set_last_error(m);
  return st;
}

#define BHIP(expr)                                                          \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess) return bfail(DL_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct Req {
  bool used = false, done = false;
  int kind = 0;  // 0 closure, 1 same generation
  int64_t n = 0, Np = 0;
  int64_t tag = 0;
  size_t off = 0, bytes = 0;  // pool region
  uint8_t* b[4] = {nullptr, nullptr, nullptr, nullptr};
  int64_t computed = 0;     // highest iterate written on the device
  int phase = 0;            // same generation: 0 = next launch is T = [P S], 1 = S' = [I + T P^T]
  std::vector<int64_t> ones;  // model sizes known on the host, ones[k] for k <= known
  int64_t iters = 0;
  int tile = 64;            // output tile of its products (Np is a multiple of it)
  bool admit_count = false; // ones[1] pending from the ingest counter
  uint64_t gen = 0;         // admission number
  int64_t icomp = 0;        // issue state: iterate the next product builds on ...
  int iphase = 0;           // ... and (same generation) which of its two products
};

// One request's product in a round, as recorded when the round was issued.
struct RoundItem {
  int slot;
  uint64_t gen;
  int kind;
  int phase;     // same generation: 0 = T = [P S], 1 = S' = [I + T P^T]
  int64_t t;     // iterate this product belongs to
  bool admit;    // this round also reads the request's admission counter
};

struct Round {
  std::vector<RoundItem> items;
  int set = 0;        // counter / descriptor / read-back set
  int64_t seq = -1;   // issue number
  bool live = false;
};

// Pool memory of a request fetched while round `after` was in flight: free
// once that round has completed.
struct Retired {
  size_t off, bytes;
  int64_t after;
};

}  // namespace

struct dl_batch {
  dl_ctx* ctx = nullptr;
  int device = 0;
  uint8_t* pool = nullptr;
  size_t pool_bytes = 0;
  std::map<size_t, size_t> free_list;  // offset -> size
  std::vector<Req> req;
  // two sets (alternating rounds) of everything a round reads or writes:
  GroupDesc* d_desc = nullptr;  // device descriptors [max] per set: the 256-, 128- and 64-tile lists in turn
  GroupDesc* h_desc = nullptr;  // pinned host descriptors, same layout (coherent, device-mapped:
                                // a kernel moves them, see move_words)
  GroupDesc* h_desc_dev = nullptr;  // device mapping of h_desc
  int* d_tot = nullptr;             // per set: live tiles of the three lists (k_group_upload)
  unsigned long long* d_cnt = nullptr;  // per set: round counters [max], then admission counters [max]
  unsigned long long* h_cnt = nullptr;  // pinned copy, same layout (coherent, device-mapped)
  unsigned long long* h_cnt_dev = nullptr;  // device mapping of h_cnt
  std::vector<unsigned long long> last;  // per set: round counters as read back in its previous round
  AdmitDesc* d_adm = nullptr;   // grouped admission descriptors [max] per set
  AdmitDesc* h_adm = nullptr;   // pinned host copy (coherent, device-mapped)
  AdmitDesc* h_adm_dev = nullptr;  // device mapping of h_adm
  hipEvent_t ev[2] = {nullptr, nullptr};  // end of each set's read-back
  std::vector<AdmitDesc> pend;  // edge-list requests admitted since the last round
  // tile table: requests with n <= tile_n[i] (the first such i) use tile_t[i]
  std::vector<int64_t> tile_n;
  std::vector<int> tile_t;
  int lookahead = 0;
  int64_t rounds_issued = 0;
  Round inflight;               // issued, not yet read (look-ahead only)
  uint64_t next_gen = 1;
  std::vector<Retired> retire;  // pool regions waiting for the round that may still read them
  int max_active = 0;
  int grid = 1024;  // persistent workgroups of the 64 and 128 tile launches
  int cus = 256;
  std::vector<int> finished;  // slots finished and not yet polled
  std::vector<int> order;     // issue_round's scratch: active slots, largest first
};

namespace {

// Output tiles by request size: 64 x 64 up to n = 256, 128 x 128 up to
// n = 1024, 256 x 256 (the direct-to-LDS kernel) above, unless the batch's
// tile table (dl_batch_tune / dl_batch_set_tiles) says otherwise.
int default_tile(int64_t n) { return n <= 256 ? 64 : (n <= 1024 ? 128 : 256); }

int tile_for(const dl_batch* b, int64_t n) {
  for (size_t i = 0; i < b->tile_n.size(); ++i)
    if (n <= b->tile_n[i]) return b->tile_t[i];
  return default_tile(n);
}

bool pool_alloc(dl_batch* b, size_t bytes, size_t* off) {
  for (auto it = b->free_list.begin(); it != b->free_list.end(); ++it) {
    if (it->second >= bytes) {
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t roff = it->first + bytes;
      b->free_list.erase(it);
      if (rest) b->free_list[roff] = rest;
      return true;
    }
  }
  return false;
}

void pool_free(dl_batch* b, size_t off, size_t bytes) {
  auto it = b->free_list.emplace(off, bytes).first;
  auto next = std::next(it);
  if (next != b->free_list.end() && it->first + it->second == next->first) {
    it->second += next->second;
    b->free_list.erase(next);
  }
  if (it != b->free_list.begin()) {
    auto prev = std::prev(it);
    if (prev->first + prev->second == it->first) {
      prev->second += it->second;
      b->free_list.erase(it);
    }
  }
}

int list_of(int tile) { return tile == 64 ? 0 : (tile == 128 ? 1 : 2); }
constexpr int kLists = 3;
int64_t pad_to(int64_t n, int t) { return (n + t - 1) / t * t; }

size_t request_bytes(int kind, int64_t Np) {
  const size_t m = (size_t)Np * Np;
  return 4 * m;  // closure: R, R^T (two each); SG: P, S (two), T
}

// Move `bytes` (a multiple of 8) from src to dst on s with k_publish; one
// side is a device mapping of coherent pinned host memory.
hipError_t move_words(const void* src, void* dst, size_t bytes, hipStream_t s) {
  return launch_publish((const unsigned long long*)src, (unsigned long long*)dst, (int)(bytes / 8), s);
}
static_assert(sizeof(GroupDesc) % 8 == 0 && sizeof(AdmitDesc) % 8 == 0, "descriptors move as 8-byte words");

// Detect the first repeat in the known model sizes.
void settle(Req& r) {
  for (int64_t k = 1; k < (int64_t)r.ones.size(); ++k)
    if (r.ones[k] == r.ones[k - 1]) {
      r.done = true;
      r.iters = k;
      return;
    }
}

}  // namespace

extern "C" {

int dl_batch_create(dl_ctx* ctx, int device, size_t pool_bytes, int max_active, dl_batch** out) {
  if (!out || pool_bytes == 0 || max_active <= 0 || max_active > kRing) return bfail(DL_EINVAL, "bad batch arguments");
  *out = nullptr;
  dl_batch* b = new (std::nothrow) dl_batch();
  if (!b) return bfail(DL_ENOMEM, "host allocation failed");
  b->ctx = ctx;
  b->device = device;
  b->max_active = max_active;
  b->req.resize(max_active);
  auto fail_destroy = [&](int st) {
    dl_batch_destroy(b);
    return st;
  };
  hipError_t e;
  if ((e = hipSetDevice(device)) != hipSuccess) return fail_destroy(bfail(DL_EHIP, "hipSetDevice"));
  if ((e = bool_kernels_init()) != hipSuccess) return fail_destroy(bfail(DL_EHIP, "kernel attributes"));
  if ((e = hipMalloc(&b->pool, pool_bytes)) != hipSuccess) {
    (void)hipGetLastError();
    return fail_destroy(bfail(DL_ENOMEM, "pool allocation failed"));
  }
  b->pool_bytes = pool_bytes;
  b->free_list[0] = pool_bytes;
  if ((e = hipMalloc(&b->d_desc, sizeof(GroupDesc) * 2 * max_active)) != hipSuccess)
    return fail_destroy(bfail(DL_ENOMEM, "descriptor allocation failed"));
  if ((e = hipMalloc(&b->d_tot, sizeof(int) * 8)) != hipSuccess)
    return fail_destroy(bfail(DL_ENOMEM, "descriptor allocation failed"));
  // host buffers the device reads or writes directly (k_publish moves them;
  // runtime copies left a gap of ~10 us before each in the kernel trace)
  constexpr unsigned kMapped = hipHostMallocMapped | hipHostMallocCoherent;
  if ((e = hipHostMalloc(&b->h_desc, sizeof(GroupDesc) * 2 * max_active, kMapped)) != hipSuccess)
    return fail_destroy(bfail(DL_ENOMEM, "pinned descriptor allocation failed"));
  if ((e = hipMalloc(&b->d_cnt, sizeof(unsigned long long) * 4 * max_active)) != hipSuccess)
    return fail_destroy(bfail(DL_ENOMEM, "counter allocation failed"));
  if ((e = hipHostMalloc(&b->h_cnt, sizeof(unsigned long long) * 4 * max_active, kMapped)) != hipSuccess)
    return fail_destroy(bfail(DL_ENOMEM, "pinned counter allocation failed"));
  if ((e = hipMemset(b->d_cnt, 0, sizeof(unsigned long long) * 4 * max_active)) != hipSuccess)
    return fail_destroy(bfail(DL_EHIP, "counter clear"));
  b->last.assign((size_t)2 * max_active, 0ull);
  if ((e = hipMalloc(&b->d_adm, sizeof(AdmitDesc) * 2 * max_active)) != hipSuccess)
    return fail_destroy(bfail(DL_ENOMEM, "admission descriptor allocation failed"));
  if ((e = hipHostMalloc(&b->h_adm, sizeof(AdmitDesc) * 2 * max_active, kMapped)) != hipSuccess)
    return fail_destroy(bfail(DL_ENOMEM, "pinned admission descriptor allocation failed"));
  if (hipHostGetDevicePointer((void**)&b->h_desc_dev, b->h_desc, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&b->h_cnt_dev, b->h_cnt, 0) != hipSuccess ||
      hipHostGetDevicePointer((void**)&b->h_adm_dev, b->h_adm, 0) != hipSuccess)
    return fail_destroy(bfail(DL_EHIP, "hipHostGetDevicePointer"));
  for (auto& ev : b->ev)
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
      return fail_destroy(bfail(DL_EHIP, "event creation failed"));
  b->pend.reserve(max_active);
  int cus = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0) cus = prop.multiProcessorCount;
  b->grid = cus * 4;
  b->cus = cus;
  *out = b;
  return DL_OK;
}

int dl_batch_destroy(dl_batch* b) {
  if (!b) return DL_OK;
  (void)hipSetDevice(b->device);
  (void)hipDeviceSynchronize();
  if (b->pool) (void)hipFree(b->pool);
  if (b->d_desc) (void)hipFree(b->d_desc);
  if (b->d_tot) (void)hipFree(b->d_tot);
  if (b->h_desc) (void)hipHostFree(b->h_desc);
  if (b->d_cnt) (void)hipFree(b->d_cnt);
  if (b->h_cnt) (void)hipHostFree(b->h_cnt);
  if (b->d_adm) (void)hipFree(b->d_adm);
  if (b->h_adm) (void)hipHostFree(b->h_adm);
  for (auto& ev : b->ev)
    if (ev) (void)hipEventDestroy(ev);
  delete b;
  return DL_OK;
}

}  // extern "C"

namespace {

// Admission shared by both submit calls: a slot, pool memory, the request's
// buffers; `fill` writes the relation into them.  A deferred admission leaves
// every device write to `fill` (which queues a grouped-admission descriptor
// that also zeroes the counter and writes S^(1) = I).
template <class Fill>
int admit(dl_batch* b, int kind, int64_t n, int64_t tag, int32_t* slot_out, hipStream_t s, bool deferred,
          Fill fill) {
  if (!b || !slot_out) return bfail(DL_EINVAL, "NULL argument");
  if (kind != 0 && kind != 1) return bfail(DL_EINVAL, "kind must be 0 (closure) or 1 (same generation)");
  if (n <= 0 || n > 16384) return bfail(DL_EINVAL, "bad relation size (1 <= n <= 16384)");
  int slot = -1;
  for (int i = 0; i < b->max_active; ++i)
    if (!b->req[i].used) {
      slot = i;
      break;
    }
  if (slot < 0) return bfail(DL_EAGAIN, "no free request slot");
  const int tile = tile_for(b, n);
  const int64_t Np = pad_to(n, tile);
  const size_t bytes = request_bytes(kind, Np);
  size_t off = 0;
  if (!pool_alloc(b, bytes, &off)) return bfail(DL_EAGAIN, "pool memory exhausted");
  BHIP(hipSetDevice(b->device));
  Req& r = b->req[slot];
  r = Req();
  r.used = true;
  r.kind = kind;
  r.n = n;
  r.Np = Np;
  r.tile = tile;
  r.tag = tag;
  r.off = off;
  r.bytes = bytes;
  uint8_t* base = b->pool + off;
  const size_t m = (size_t)Np * Np;
  r.ones.push_back(0);
  r.gen = b->next_gen++;
  // admission counter, read back by the next round, which uses counter set
  // rounds_issued % 2 (the round in flight, if any, uses the other set)
  unsigned long long* adm = b->d_cnt + (size_t)(b->rounds_issued & 1) * 2 * b->max_active + b->max_active + slot;
  if (kind == 0) {
    for (int i = 0; i < 4; ++i) r.b[i] = base + m * i;  // R0, R0T, R1, R1T
    if (!deferred) BHIP(launch_ring_clear(adm, nullptr, 0, 1, 0, s));
    // R^(1) = A and R^(1)T = A^T + I: a squaring step computes
    // [R (R^T + I)^T] = [R R + R] (= [A + R R] along the iteration) and
    // writes the next R^T + I as its transposed output
    int rc = fill(n, Np, (int8_t*)base, (int8_t*)r.b[2], (int8_t*)r.b[3], adm);
    if (rc) {
      pool_free(b, off, bytes);
      r = Req();
      return rc;
    }
    r.computed = r.icomp = 1;
    r.admit_count = true;
  } else {
    for (int i = 0; i < 4; ++i) r.b[i] = base + m * i;  // P, S0, S1, T
    int rc = fill(n, Np, (int8_t*)base, (int8_t*)r.b[0], nullptr, nullptr);
    if (rc) {
      pool_free(b, off, bytes);
      r = Req();
      return rc;
    }
    if (!deferred) BHIP(launch_identity(P_I8, r.b[2], (int)Np, (int)n, s));
    r.computed = r.icomp = 1;
    r.ones.push_back(n);  // S^(1) = I: one fact diag(x, x) per constant
  }
  *slot_out = slot;
  return DL_OK;
}

}  // namespace

extern "C" {

int dl_batch_submit(dl_batch* b, int kind, int64_t n, const uint8_t* A, int64_t lda, int64_t tag, int32_t* slot_out,
                    void* stream) {
  if (!A || lda < n) return bfail(DL_EINVAL, "bad relation (A NULL or lda < n)");
  hipStream_t s = (hipStream_t)stream;
  return admit(b, kind, n, tag, slot_out, s, false,
               [&](int64_t nn, int64_t Np, int8_t* base, int8_t* M, int8_t* MT, unsigned long long* ones) -> int {
                 // closure: M = R^(1), MT = R^(1)T + I; same generation: M = P
                 (void)base;
                 BHIP(launch_ingest(P_I8, A, lda, (int)nn, (int)Np, nullptr, nullptr, M, MT, kind == 0 ? 2 : 0, ones, s));
                 return DL_OK;
               });
}

int dl_batch_submit_edges(dl_batch* b, int kind, int64_t n, const int32_t* edges, int64_t m, int64_t tag,
                          int32_t* slot_out, void* stream) {
  if (m < 0 || (m > 0 && !edges)) return bfail(DL_EINVAL, "bad edge list");
  (void)stream;  // the device work runs in the next dl_batch_step, on its stream
  return admit(b, kind, n, tag, slot_out, nullptr, true,
               [&](int64_t nn, int64_t Np, int8_t* base, int8_t* M, int8_t* MT, unsigned long long* ones) -> int {
                 const long long mb = (long long)Np * Np;
                 // the request's buffers are contiguous from base (closure:
                 // R0, R0T, R1, R1T; same generation: P, S0, S1, T).  Closure
                 // clears R1 and R1T = I (before the edges' A^T), the first
                 // iterate: the first product writes every byte of R0 and R0T.
                 // Same generation clears P, S0 and S1 = I (S0, which its
                 // first S' product writes whole, lies between the other two).
                 AdmitDesc a{};
                 a.base = kind == 0 ? base + 2 * mb : base;
                 a.clear_units = (kind == 0 ? 2 : 3) * mb / 16;
                 a.ident_off = kind == 0 ? mb : 2 * mb;
                 a.M = M;
                 a.M2 = nullptr;
                 a.MT = MT;
                 a.ones = ones;
                 a.edges = edges;
                 a.m = m;
                 a.n = (int)nn;
                 a.Np = (int)Np;
                 b->pend.push_back(a);
                 return DL_OK;
               });
}

int dl_batch_submit_edges_n(dl_batch* b, int32_t count, const int32_t* kinds, const int64_t* ns,
                            const int32_t* const* edges, const int64_t* ms, const int64_t* tags, int32_t* slots,
                            int32_t* admitted, void* stream) {
  if (!admitted) return bfail(DL_EINVAL, "NULL admitted");
  *admitted = 0;
  if (count < 0 || (count > 0 && (!kinds || !ns || !edges || !ms || !tags || !slots)))
    return bfail(DL_EINVAL, "bad request arrays");
  for (int32_t i = 0; i < count; ++i) {
    const int rc = dl_batch_submit_edges(b, kinds[i], ns[i], edges[i], ms[i], tags[i], slots + i, stream);
    if (rc == DL_EAGAIN) return DL_OK;  // the first request that does not fit ends the call
    if (rc) return rc;
    *admitted = i + 1;
  }
  return DL_OK;
}

}  // extern "C"

namespace {

// Enqueue one round on s: the grouped admission of pending edge-list
// requests, then one product for every unfinished request (as far as the
// host knows), then the read-back of the round's counters into its set.
// rd is left not live when there was nothing to run.
int issue_round(dl_batch* b, hipStream_t s, Round& rd) {
  rd.items.clear();
  rd.live = false;
  const int set = (int)(b->rounds_issued & 1);
  const int M = b->max_active;
  // edge-list requests admitted since the last round: one clear and one
  // scatter launch for all of them, ahead of their first product
  if (!b->pend.empty()) {
    const int na = (int)b->pend.size();
    AdmitDesc* ha = b->h_adm + (size_t)set * M;
    AdmitDesc* da = b->d_adm + (size_t)set * M;
    long long units = 0, edges = 0;
    for (int i = 0; i < na; ++i) {
      AdmitDesc& a = b->pend[i];
      a.clear_start = units;
      a.edge_start = edges;
      units += a.clear_units;
      edges += a.m;
      ha[i] = a;
    }
    b->pend.clear();
    BHIP(move_words(b->h_adm_dev + (size_t)set * M, da, sizeof(AdmitDesc) * na, s));
    BHIP(launch_admit(da, na, units, edges, s));
  }
  // this round's work lists (256, 128 and 64 tiles, one after the other in
  // the set's descriptors); the counter of a request's product is
  // d_cnt[set][slot]
  unsigned long long* cnt = b->d_cnt + (size_t)set * 2 * M;
  // With the previous round still in flight, a request's product there may
  // turn out to be its last: its counter in that round's set then equals the
  // value read after that set's previous round plus the model size the host
  // already holds for the iterate before.  The device tests this before this
  // round's products (k_group_upload).
  const bool ahead = b->lookahead && b->inflight.live && b->inflight.seq == b->rounds_issued - 1;
  const unsigned long long* pcnt = b->d_cnt + (size_t)(set ^ 1) * 2 * M;
  const unsigned long long* plast = b->last.data() + (size_t)(set ^ 1) * M;
  GroupDesc* hset = b->h_desc + (size_t)set * M;
  GroupDesc* dset = b->d_desc + (size_t)set * M;
  int na[kLists] = {0, 0, 0}, tiles[kLists] = {0, 0, 0};
  // the largest requests first: a tile's time grows with Np (its K loop),
  // and the persistent workgroups take the list in passes, so the short
  // tiles of small requests fill the last pass (largest-first scheduling)
  std::vector<int>& order = b->order;
  order.clear();
  for (int i = 0; i < M; ++i) {
    const Req& r = b->req[i];
    if (!r.used || r.done) continue;
    ++na[list_of(r.tile)];
    order.push_back(i);
  }
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->req[x].Np > b->req[y].Np; });
  int first[kLists], fill[kLists] = {0, 0, 0};
  first[2] = 0;
  first[1] = na[2];
  first[0] = na[2] + na[1];
  for (const int i : order) {
    Req& r = b->req[i];
    const int li = list_of(r.tile);
    GroupDesc& g = hset[first[li] + fill[li]];
    std::memset(&g, 0, sizeof g);
    g.Np = (int)r.Np;
    g.n_valid = (int)r.n;
    g.tile_start = tiles[li];
    g.cnt = nullptr;
    RoundItem it{i, r.gen, r.kind, r.iphase, r.icomp + 1, r.admit_count};
    r.admit_count = false;
    const int64_t t = r.icomp + 1;  // iterate this product belongs to
    // the previous round made iterate t - 1 (closure, or same generation's
    // S' before a T product) and the host knows the size of iterate t - 2
    if (ahead && (r.kind == 0 || r.iphase == 0) && t >= 3 && (int64_t)r.ones.size() > t - 2) {
      g.chk = pcnt + i;
      g.chk_val = plast[i] + (unsigned long long)r.ones[(size_t)(t - 2)];
    }
    if (r.kind == 0) {
      const int prev = (int)((t - 1) & 1), cur = (int)(t & 1);
      g.X = r.b[2 * prev];
      g.Y = r.b[2 * prev + 1];
      g.outT_ident = 1;  // the next step's right operand R^T + I
      g.out = r.b[2 * cur];
      g.outT = r.b[2 * cur + 1];
      g.cnt = cnt + i;
      r.icomp = t;
    } else if (r.iphase == 0) {
      const int prev = (int)((t - 1) & 1);
      g.X = r.b[0];
      g.Y = r.b[1 + prev];
      g.out = r.b[3];
      r.iphase = 1;
    } else {
      const int cur = (int)(t & 1);
      g.X = r.b[3];
      g.Y = r.b[0];
      g.add_identity = 1;
      g.out = r.b[1 + cur];
      g.cnt = cnt + i;
      // S' is symmetric: only the tiles tm <= tn, mirrored
      g.sym = 1;
      r.icomp = t;
      r.iphase = 0;
    }
    const int tside = (int)(r.Np / r.tile);
    tiles[li] += g.sym ? tside * (tside + 1) / 2 : tside * tside;
    rd.items.push_back(it);
    ++fill[li];
  }
  if (rd.items.empty()) return DL_OK;
  // descriptor segments in array order: the 256-, 128- and 64-tile lists
  GroupLists gl{{0, na[2], na[2] + na[1], na[2] + na[1] + na[0]}, {256, 128, 64}};
  int* tot = b->d_tot + 4 * set;
  BHIP(launch_group_upload(b->h_desc_dev + (size_t)set * M, dset, gl, tot, s));
  for (int li = kLists - 1; li >= 0; --li) {  // the largest tiles first
    if (!na[li]) continue;
    const int grid = li == 2 ? b->cus : b->grid;  // the 256 tiles take a whole CU each
    BHIP(launch_group_step(64 << li, dset + first[li], na[li], tiles[li], std::min(grid, tiles[li]), s,
                           tot + (2 - li)));
  }
  // round and admission counters of the set in one read-back
  BHIP(move_words(cnt, b->h_cnt_dev + (size_t)set * 2 * M, sizeof(unsigned long long) * 2 * M, s));
  BHIP(hipEventRecord(b->ev[set], s));
  rd.set = set;
  rd.seq = b->rounds_issued;
  rd.live = true;
  ++b->rounds_issued;
  return DL_OK;
}

// Wait for a round's read-back and take its model sizes; entries of requests
// already finished or fetched (and their slots reused) are skipped.
int complete_round(dl_batch* b, Round& rd, int* finished) {
  if (!rd.live) return DL_OK;
  BHIP(hipEventSynchronize(b->ev[rd.set]));
  rd.live = false;
  const int M = b->max_active;
  const unsigned long long* hc = b->h_cnt + (size_t)rd.set * 2 * M;
  unsigned long long* last = b->last.data() + (size_t)rd.set * M;
  for (const RoundItem& it : rd.items) {
    Req& r = b->req[it.slot];
    if (!r.used || r.gen != it.gen || r.done) continue;
    if (it.admit) r.ones.push_back((int64_t)hc[M + it.slot]);  // ones[1] = |A|
    const int64_t ones = (int64_t)(hc[it.slot] - last[it.slot]);  // this round's product
    if (it.kind == 0) {
      r.computed = it.t;
      r.ones.push_back(ones);
    } else if (it.phase == 0) {
      r.phase = 1;
    } else {
      r.computed = it.t;
      r.phase = 0;
      r.ones.push_back(ones);
    }
    settle(r);
    if (r.done) {
      b->finished.push_back(it.slot);
      ++*finished;
    }
  }
  std::copy(hc, hc + M, last);
  return DL_OK;
}

}  // namespace

extern "C" {

int dl_batch_set_lookahead(dl_batch* b, int32_t rounds) {
  if (!b) return bfail(DL_EINVAL, "NULL batch");
  if (rounds != 0 && rounds != 1) return bfail(DL_EINVAL, "look-ahead must be 0 or 1 rounds");
  if (rounds == 0 && b->inflight.live) return bfail(DL_EINVAL, "a round is in flight: step until none is");
  b->lookahead = rounds;
  return DL_OK;
}

int dl_batch_step(dl_batch* b, int32_t* active_out, int32_t* finished_out, void* stream) {
  if (!b) return bfail(DL_EINVAL, "NULL batch");
  hipStream_t s = (hipStream_t)stream;
  BHIP(hipSetDevice(b->device));
  int finished = 0, rc = DL_OK;
  Round next;
  if ((rc = issue_round(b, s, next))) return rc;
  int64_t done_seq = -1;  // rounds up to this one have completed
  if (b->lookahead == 0) {
    done_seq = next.seq;
    rc = complete_round(b, next, &finished);
  } else {
    // wait for the round issued by the previous call while `next` runs
    done_seq = b->inflight.live ? b->inflight.seq : -1;
    rc = complete_round(b, b->inflight, &finished);
    b->inflight = std::move(next);
  }
  if (rc) return rc;
  // pool memory fetched while a now completed round was in flight is free
  // (the round just issued skipped those requests: their slots were empty)
  size_t kept = 0;
  for (const Retired& q : b->retire) {
    if (q.after <= done_seq)
      pool_free(b, q.off, q.bytes);
    else
      b->retire[kept++] = q;
  }
  b->retire.resize(kept);
  int active = 0;
  for (int i = 0; i < b->max_active; ++i) active += b->req[i].used && !b->req[i].done;
  if (active_out) *active_out = active;
  if (finished_out) *finished_out = finished;
  return DL_OK;
}

int dl_batch_poll(dl_batch* b, int64_t* tags, int32_t* slots, int32_t* iters, int32_t cap, int32_t* count) {
  if (!b || !count || cap < 0) return bfail(DL_EINVAL, "bad poll arguments");
  int c = 0;
  while (c < cap && !b->finished.empty()) {
    const int sl = b->finished.front();
    b->finished.erase(b->finished.begin());
    if (tags) tags[c] = b->req[sl].tag;
    if (slots) slots[c] = sl;
    if (iters) iters[c] = (int32_t)b->req[sl].iters;
    ++c;
  }
  *count = c;
  return DL_OK;
}

int dl_batch_fetch(dl_batch* b, int32_t slot, uint8_t* R, int64_t ldr, int64_t* ones_out, void* stream) {
  if (!b || slot < 0 || slot >= b->max_active || !b->req[slot].used) return bfail(DL_EINVAL, "bad slot");
  Req& r = b->req[slot];
  if (!r.done) return bfail(DL_EINVAL, "request not finished");
  if (R && ldr < r.n) return bfail(DL_EINVAL, "ldr < n");
  hipStream_t s = (hipStream_t)stream;
  BHIP(hipSetDevice(b->device));
  if (R) {
    // the fixpoint iterate r.iters lives in buffer r.iters % 2 of its kind
    const uint8_t* src = r.kind == 0 ? r.b[2 * (int)(r.iters & 1)] : r.b[1 + (int)(r.iters & 1)];
    BHIP(launch_emit(P_I8, src, (int)r.Np, 0, (int)r.n, R, ldr, s));
    BHIP(hipStreamSynchronize(s));
  }
  if (ones_out) *ones_out = r.ones[r.iters];
  // a request fetched before it was polled is no longer reported by dl_batch_poll
  b->finished.erase(std::remove(b->finished.begin(), b->finished.end(), slot), b->finished.end());
  if (b->inflight.live)
    b->retire.push_back({r.off, r.bytes, b->inflight.seq});  // the round in flight may still read it
  else
    pool_free(b, r.off, r.bytes);
  r = Req();
  return DL_OK;
}

int dl_batch_release_n(dl_batch* b, int32_t count, const int32_t* slots, int64_t* ones) {
  if (count < 0 || (count > 0 && !slots)) return bfail(DL_EINVAL, "bad slot array");
  for (int32_t i = 0; i < count; ++i) {
    const int rc = dl_batch_fetch(b, slots[i], nullptr, 0, ones ? ones + i : nullptr, nullptr);
    if (rc) return rc;
  }
  return DL_OK;
}

int dl_batch_set_tiles(dl_batch* b, const int64_t* sizes, const int32_t* tiles, int32_t k) {
  if (!b || k < 0 || (k > 0 && (!sizes || !tiles))) return bfail(DL_EINVAL, "bad tile table");
  for (int i = 0; i < k; ++i) {
    if (sizes[i] <= 0 || (i > 0 && sizes[i] <= sizes[i - 1])) return bfail(DL_EINVAL, "sizes must ascend");
    if (tiles[i] != 64 && tiles[i] != 128 && tiles[i] != 256) return bfail(DL_EINVAL, "tiles are 64, 128 or 256");
  }
  b->tile_n.assign(sizes, sizes + k);
  b->tile_t.assign(tiles, tiles + k);
  return DL_OK;
}

int dl_batch_tune(dl_batch* b, const int64_t* sizes_in, int32_t k, int32_t* tiles_out, double* ms_out,
                  void* stream) {
  static const int64_t kSizes[] = {96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048};
  if (!b || k < 0 || (k > 0 && !sizes_in)) return bfail(DL_EINVAL, "bad size list");
  const int64_t* sizes = k > 0 ? sizes_in : kSizes;
  const int ns = k > 0 ? k : (int)(sizeof kSizes / sizeof kSizes[0]);
  for (int i = 0; i < ns; ++i)
    if (sizes[i] <= 0 || sizes[i] > 16384 || (i > 0 && sizes[i] <= sizes[i - 1]))
      return bfail(DL_EINVAL, "sizes must ascend within 1 .. 16384");
  hipStream_t s = (hipStream_t)stream;
  BHIP(hipSetDevice(b->device));
  static const int kTiles[3] = {64, 128, 256};
  constexpr int kRounds = 3;
  std::vector<int32_t> choice(ns);
  std::vector<double> times((size_t)3 * ns, -1.0);
  hipEvent_t ea = nullptr, eb = nullptr;
  BHIP(hipEventCreate(&ea));
  if (hipEventCreate(&eb) != hipSuccess) {
    (void)hipEventDestroy(ea);
    return bfail(DL_EHIP, "hipEventCreate");
  }
  uint8_t* buf = nullptr;
  size_t buf_bytes = 0;
  int rc = DL_OK;
  for (int si = 0; si < ns && rc == DL_OK; ++si) {
    const int64_t n = sizes[si];
    // the same requests for every tile size: about eight 2048-sized
    // products of work, 1 .. 256 requests
    const double want = 8.0 * 2048.0 * 2048.0 * 2048.0 / ((double)n * n * n);
    const int count = (int)std::min(256.0, std::max(1.0, std::floor(want)));
    const int64_t npmax = pad_to(n, 256);
    const size_t req = 4 * (size_t)npmax * npmax;
    const size_t need = (size_t)count * req + (size_t)count * sizeof(GroupDesc) + 256;
    if (need > buf_bytes) {
      if (buf) (void)hipFree(buf);
      buf = nullptr;
      buf_bytes = 0;
      if (hipMalloc(&buf, need) != hipSuccess) {
        (void)hipGetLastError();
        rc = bfail(DL_ENOMEM, "temporary memory for the tile autotuner");
        break;
      }
      buf_bytes = need;
    }
    GroupDesc* ddesc = (GroupDesc*)(buf + (size_t)count * req);
    unsigned long long* dcnt = (unsigned long long*)(ddesc + count);
    std::vector<double> med(3, -1.0);
    std::vector<std::vector<double>> samp(3);
    std::vector<GroupDesc> h((size_t)count);
    for (int round = 0; round <= kRounds && rc == DL_OK; ++round) {  // round 0 warms up
      for (int ti = 0; ti < 3 && rc == DL_OK; ++ti) {
        const int T = kTiles[ti];
        const int64_t Np = pad_to(n, T);
        const size_t m = (size_t)Np * Np;
        int tiles = 0;
        for (int q = 0; q < count; ++q) {
          uint8_t* base = buf + (size_t)q * req;
          GroupDesc& g = h[q];
          std::memset(&g, 0, sizeof g);
          g.X = base;
          g.Y = base + m;
          g.outT_ident = 1;
          g.out = base + 2 * m;
          g.outT = base + 3 * m;
          g.cnt = dcnt;
          g.Np = (int)Np;
          g.n_valid = (int)n;
          g.tile_start = tiles;
          tiles += (int)((Np / T) * (Np / T));
          if (round == 0) {  // pseudo-random 0/1 operands
            hipError_t e = launch_hash_bool(base, Np, (int)n, (int)Np, 11u + (unsigned)q, s);
            if (e == hipSuccess) e = launch_hash_bool(base + m, Np, (int)n, (int)Np, 977u + (unsigned)q, s);
            if (e != hipSuccess) {
              rc = bfail(DL_EHIP, "autotuner operands");
              break;
            }
          }
        }
        if (rc) break;
        hipError_t e = hipMemcpyAsync(ddesc, h.data(), sizeof(GroupDesc) * count, hipMemcpyHostToDevice, s);
        const int grid = std::min(T == 256 ? b->cus : b->grid, tiles);
        const int reps = round == 0 ? 1 : 3;
        if (e == hipSuccess) e = hipEventRecord(ea, s);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_group_step(T, ddesc, count, tiles, grid, s);
        if (e == hipSuccess) e = hipEventRecord(eb, s);
        if (e == hipSuccess) e = hipEventSynchronize(eb);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, ea, eb);
        if (e != hipSuccess) {
          rc = bfail(DL_EHIP, std::string("autotuner launches: ") + hipGetErrorString(e));
          break;
        }
        if (round > 0) samp[ti].push_back((double)t / reps / count);  // ms per request-product
      }
    }
    if (rc) break;
    int best = -1;
    for (int ti = 0; ti < 3; ++ti) {
      std::sort(samp[ti].begin(), samp[ti].end());
      med[ti] = samp[ti][samp[ti].size() / 2];
      times[(size_t)3 * si + ti] = med[ti];
      if (best < 0 || med[ti] < med[best]) best = ti;
    }
    // keep the built-in choice unless another tile beats it by more than 5%
    const int def = list_of(default_tile(n));
    choice[si] = med[def] <= 1.05 * med[best] ? kTiles[def] : kTiles[best];
  }
  (void)hipEventDestroy(ea);
  (void)hipEventDestroy(eb);
  if (buf) {
    (void)hipStreamSynchronize(s);
    (void)hipFree(buf);
  }
  if (rc) return rc;
  b->tile_n.assign(sizes, sizes + ns);
  b->tile_t.assign(choice.begin(), choice.end());
  if (tiles_out) std::copy(choice.begin(), choice.end(), tiles_out);
  if (ms_out) std::copy(times.begin(), times.end(), ms_out);
  return DL_OK;
}

int dl_batch_info(dl_batch* b, int32_t* active, int32_t* used_slots, size_t* pool_free_bytes) {
  if (!b) return bfail(DL_EINVAL, "NULL batch");
  int act = 0, used = 0;
  for (auto& r : b->req) {
    used += r.used;
    act += r.used && !r.done;
  }
  size_t fr = 0;
  for (auto& kv : b->free_list) fr += kv.second;
  if (active) *active = act;
  if (used_slots) *used_slots = used;
  if (pool_free_bytes) *pool_free_bytes = fr;
  return DL_OK;
}

}  // extern "C"
