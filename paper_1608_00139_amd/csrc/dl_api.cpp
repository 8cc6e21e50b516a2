// dl_api.cpp -- the C ABI of include/dl.h: argument checks, workspace, and the
// fixpoint driver that enqueues step launches and reads back model sizes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <climits>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/dl.h"
#include "common.h"
#include "ctx.h"
#include "eps_solve.h"

using namespace dl;

namespace {

thread_local std::string g_last_error;

int fail(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

int hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return DL_EHIP;
}

#define DL_HIP(expr)                                      \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return hip_fail(e_, #expr);     \
  } while (0)

}  // namespace

namespace dl {
void set_last_error(const std::string& m) { g_last_error = m; }

int tuned_config(const dl_ctx* c, int prec, int64_t np) {
  for (const auto& t : c->tuned)
    if (t.prec == prec && t.np == np) return t.cfg;
  return -1;
}

int pick_config(const dl_ctx* c, int prec, int64_t np) {
  const int t = tuned_config(c, prec, np);
  return (t >= 0 && t != kCfgWholeFixpoint) ? t : choose_nt_config(prec, np);
}
}  // namespace dl


namespace {

int ensure_ws(dl_ctx* c, size_t need) {
  if (need <= c->ws_size) return DL_OK;
  if (c->budget && need > c->budget)
    return fail(DL_ENOMEM, "workspace of " + std::to_string(need) + " bytes exceeds the budget of " +
                               std::to_string(c->budget));
  if (c->ws) {
    hipError_t e = hipFree(c->ws);
    c->ws = nullptr;
    c->ws_size = 0;
    if (e != hipSuccess) return hip_fail(e, "hipFree(workspace)");
  }
  hipError_t e = hipMalloc(&c->ws, need);
  if (e != hipSuccess) {
    c->ws = nullptr;
    (void)hipGetLastError();
    return fail(DL_ENOMEM, "hipMalloc of " + std::to_string(need) + " bytes failed");
  }
  c->ws_size = need;
  return DL_OK;
}

bool overlaps(const void* a, size_t alen, const void* b, size_t blen) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + blen && y < x + alen;
}

size_t mat_span(int64_t n, int64_t ld) { return n <= 0 ? 0 : (size_t)((n - 1) * ld + n); }

int check_common(dl_ctx* ctx, int64_t n, const void* in, int64_t ldin, const void* out, int64_t ldout) {
  if (!ctx) return fail(DL_EINVAL, "ctx is NULL");
  if (n < 0) return fail(DL_EINVAL, "n < 0");
  if (n > (1 << 16)) return fail(DL_EINVAL, "n > 65536 is not supported");
  if (n == 0) return DL_OK;
  if (!in || !out) return fail(DL_EINVAL, "NULL matrix pointer");
  if (ldin < n || ldout < n) return fail(DL_EINVAL, "leading dimension smaller than n");
  if (overlaps(in, mat_span(n, ldin), out, mat_span(n, ldout)))
    return fail(DL_EINVAL, "output overlaps the input");
  return DL_OK;
}

int set_device(dl_ctx* c) {
  DL_HIP(hipSetDevice(c->device));
  return DL_OK;
}

// Timed launch bracket (events only when timing is on).  Brackets take pairs
// from the context's pool in order; the launches that did work are queued in
// ctx->pending and their times are read only when the statistics are asked
// for (or the pool grows large), so a timed run does not wait on
// elapsed-time queries between calls.
constexpr size_t kMaxPendingEvents = 4096;

void resolve_timing(dl_ctx* c) {
  for (auto& m : c->pending) {
    float t = 0.f;
    const EventPair& ep = c->events[m.second];
    if (hipEventSynchronize(ep.b) == hipSuccess && hipEventElapsedTime(&t, ep.a, ep.b) == hipSuccess) {
      c->ms[m.first] += t;
      c->launches[m.first] += 1;
    }
  }
  c->pending.clear();
  c->ev_cursor = 0;
}

struct Timer {
  dl_ctx* c;
  hipStream_t s;
  std::vector<std::pair<int, int>> marks;  // (class, event index)
  int begin(int cls) {
    if (!c->timing) return -1;
    if (c->ev_cursor >= c->events.size()) {
      EventPair ep;
      if (hipEventCreate(&ep.a) != hipSuccess || hipEventCreate(&ep.b) != hipSuccess) return -1;
      c->events.push_back(ep);
    }
    const int idx = (int)c->ev_cursor++;
    (void)hipEventRecord(c->events[idx].a, s);
    marks.push_back({cls, idx});
    return idx;
  }
  void end(int idx) {
    if (idx >= 0) (void)hipEventRecord(c->events[idx].b, s);
  }
  // Queue the first `keep` marks of class cls (launches that did work).
  void collect(int cls, int64_t keep) {
    int64_t taken = 0;
    for (auto& m : marks) {
      if (m.first != cls) continue;
      if (taken >= keep) break;
      c->pending.push_back(m);
      ++taken;
    }
  }
};

enum Mode { M_PLAIN = 0, M_SQUARE = 1, M_SG = 2 };

// Workspace of one fixpoint: four operand-precision matrices.
size_t fix_ws_bytes(int prec, int64_t Np) { return 4 * (size_t)mat_bytes(prec, Np) + 256; }

// Device and pinned host state of one fixpoint in flight.
struct FixSlot {
  uint8_t* ws = nullptr;
  unsigned long long* ring = nullptr;    // device ring of model sizes
  int* conv = nullptr;                   // device convergence step
  unsigned long long* h_ring = nullptr;  // pinned copies read after `ev`
  unsigned long long* h_ring_dev = nullptr;  // device mapping of h_ring
  int* h_conv = nullptr;
  hipEvent_t ev = nullptr;
};

// One fixpoint: ingest, chunks of step launches with device-side early exit,
// emit.  After each chunk the ring and the convergence step are copied to
// pinned memory and the slot's event is recorded; advance() reads them once
// that event has completed and enqueues the next chunk or the emit.  Nothing
// here waits on the device, so a driver can keep several fixpoints in flight
// on one stream and read one back while the device runs another's products.
class Fix {
 public:
  Fix(dl_ctx* c, const FixSlot& sl, int mode, int64_t n, const uint8_t* A, int64_t lda, uint8_t* R, int64_t ldr,
      int prec, int32_t max_steps, hipStream_t s)
      : c_(c), sl_(sl), mode_(mode), n_(n), A_(A), lda_(lda), R_(R), ldr_(ldr), prec_(prec),
        max_steps_(max_steps), s_(s), tm_{c, s, {}} {}

  bool done() const { return done_; }
  const FixSlot& slot() const { return sl_; }

  // Ingest and the first chunk, or straight to the emit when max_steps <= 1
  // needs no product.
  int start() {
    Np_ = padded_size_for(prec_, n_);
    cfg_ = pick_config(c_, prec_, Np_);
    const size_t matT = (size_t)mat_bytes(prec_, Np_);
    uint8_t* op[4];
    for (int i = 0; i < 4; ++i) op[i] = sl_.ws + i * matT;
    // the whole ring, so that chunks need no clear until the steps wrap
    DL_HIP(launch_ring_clear(sl_.ring, sl_.conv, 0, kRing, 1, s_));
    // The closure steps add the previous iterate instead of A (plain: A^T),
    // which gives the same iterates: R^(k) = A + f(R^(k-1)) lies inside
    // A + f(R^(k)) because f is monotone and R^(k-1) <= R^(k), and it
    // contains A; so A + f(R^(k)) = R^(k) + f(R^(k)).  That sum is one
    // product once the right operand carries the identity: R R + R =
    // R (R + I) for squaring (Y = R^T + I, written by each step as its
    // transposed output), S A^T + S = S (A + I)^T for the plain series
    // (Y = A + I, written at ingest); no addend is read.
    if (mode_ == M_PLAIN) {
      // state S = R^T; S^(1) = A^T; product operand Y = A + I
      Yop_ = op[0];
      S_[0] = op[1];
      S_[1] = op[2];
      DL_HIP(launch_ingest(prec_, A_, lda_, (int)n_, (int)Np_, nullptr, nullptr, Yop_, S_[1], 1, sl_.ring + 1, s_));
    } else if (mode_ == M_SQUARE) {
      // R^(1) = A and R^(1)T + I
      S_[0] = op[0];
      ST_[0] = op[1];
      S_[1] = op[2];
      ST_[1] = op[3];
      DL_HIP(launch_ingest(prec_, A_, lda_, (int)n_, (int)Np_, nullptr, nullptr, S_[1], ST_[1], 2, sl_.ring + 1, s_));
    } else {
      // P in operand precision; S^(1) = I; intermediate T
      Yop_ = op[0];
      S_[0] = op[1];
      S_[1] = op[2];
      Tmp_ = op[3];
      DL_HIP(launch_ingest(prec_, A_, lda_, (int)n_, (int)Np_, nullptr, nullptr, Yop_, nullptr, 0, nullptr, s_));
      DL_HIP(launch_identity(prec_, S_[1], (int)Np_, (int)n_, s_));
      DL_HIP(launch_ring_set(sl_.ring, 1, (unsigned long long)n_, s_));
      // S' is symmetric: its product runs on the upper-triangle tiles only,
      // split stream-K over the compute units (scratch after the operands)
      if (sk_supported(prec_, cfg_, Np_)) {
        sk_plan(Np_, skq_);
        skq_.scratch = sl_.ws + 4 * matT;
        skq_.tile_cnt = (unsigned*)(skq_.scratch + (size_t)skq_.tiles * skq_.maxc * 65536);
        DL_HIP(hipMemsetAsync(skq_.tile_cnt, 0, (size_t)skq_.tiles * sizeof(unsigned), s_));
        use_sk_ = true;
      }
    }
    // When the caller's R has exactly the layout of an int8 iterate (no
    // padding, row stride Np, not transposed), it serves as iterate buffer
    // S[0]: the confirming step writes an iterate equal to the one before
    // it, so at a confirmed fixpoint both buffers hold the model and no
    // emit is needed.
    if (prec_ == P_I8 && mode_ != M_PLAIN && n_ == Np_ && ldr_ == Np_ && (uintptr_t)R_ % 256 == 0) {
      S_[0] = R_;
      r_is_s0_ = true;
    }
    const TileCfg tc = nt_config(prec_, cfg_);
    p_.ld = Np_;
    p_.Np = (int)Np_;
    p_.n_valid = (int)n_;
    p_.ones = sl_.ring;
    p_.conv = sl_.conv;
    p_.tiles_m = (int)(Np_ / tc.bm);
    p_.tiles_n = (int)(Np_ / tc.bn);
    computed_ = max_steps_ >= 1 ? 1 : 0;
    if (max_steps_ == 1) return readback(1);  // step 1 came from ingest; one read-back settles it
    if (max_steps_ >= 2) return chunk();
    return emit();
  }

  // The slot's event has completed: take the counts of the last chunk.
  int advance() {
    const int cv = sl_.h_conv[0];
    const int64_t upto = pending_;
    int64_t last = upto;
    if (cv != kNotConverged) last = std::min<int64_t>(last, cv);
    const int64_t first = (int64_t)ones_.size() - 1;  // slot 1 may be unread yet
    if ((int64_t)ones_.size() < last + 1) ones_.resize(last + 1, 0);
    for (int64_t k = std::max<int64_t>(1, first); k <= last; ++k) ones_[k] = (int64_t)sl_.h_ring[k % kRing];
    if (cv != kNotConverged) {
      iters_ = cv;
    } else if (upto >= 1 && ones_[upto] == ones_[upto - 1]) {
      iters_ = upto;
    }
    computed_ = (iters_ >= 0) ? iters_ : upto;
    if (iters_ < 0 && s0_ <= max_steps_) return chunk();
    return emit();
  }

  // After the stream has been synchronised: timing and the caller's outputs.
  void finish(int64_t* ones_out, int32_t* steps_out, int32_t* converged_out) {
    const int64_t last = computed_;
    if (c_->timing) {
      // the timed launches (one per chunk) did work when some product did:
      // steps 2 .. computed
      tm_.collect(0, last >= 2 ? (last - 1) : 0);
    }
    if (ones_out) {
      for (int64_t k = 0; k <= last; ++k) ones_out[k] = k < (int64_t)ones_.size() ? ones_[k] : 0;
      if (last == 0) ones_out[0] = 0;
    }
    if (steps_out) *steps_out = (int32_t)last;
    if (converged_out) *converged_out = iters_ >= 0 ? 1 : 0;
  }

 private:
  // Chunk sizes: squaring needs 2 + log2(D) steps (at most 18 for n <=
  // 65536): a first chunk of 6 covers D <= 16, then 4, 8, ...; launches
  // after the fixpoint return at once but still cost a few microseconds
  // each.  The plain series starts at 4 and doubles; the same-generation
  // series (two launches a step, each ~3 us when it returns at once) starts
  // at 4 and grows by half, so that fewer steps run past its fixpoint.
  int chunk() {
    if (chunk_ == 0) chunk_ = mode_ == M_SQUARE ? 6 : 4;
    const int cnt = (int)std::min<int64_t>(chunk_, (int64_t)max_steps_ - s0_ + 1);
    // entries of steps >= kRing still hold the counts of kRing steps before
    if (s0_ + cnt > kRing) DL_HIP(launch_ring_clear(sl_.ring, sl_.conv, (int)s0_, cnt, 0, s_));
    for (int64_t t = s0_; t < s0_ + cnt; ++t) {
      const int prev = (int)((t - 1) & 1), cur = (int)(t & 1);
      NTParams& p = p_;
      p.step = (int)t;
      p.add = nullptr;
      p.outT_ident = 0;
      // timing samples the chunk's first product: it always does work (the
      // chunk exists because the last read-back showed no repeat, except
      // for an empty relation, which finish() leaves uncounted), and the
      // others run back to back (events between launches cost ~10 us each)
      const bool timed = t == s0_;
      if (mode_ == M_PLAIN) {
        p.X = S_[prev]; p.Y = Yop_; p.add_identity = 0;
        p.out = S_[cur]; p.outT = nullptr; p.count = 1; p.check = 1;
        int ev = timed ? tm_.begin(0) : -1;
        DL_HIP(launch_nt_step(prec_, cfg_, p, s_));
        tm_.end(ev);
      } else if (mode_ == M_SQUARE) {
        p.X = S_[prev]; p.Y = ST_[prev]; p.add_identity = 0;
        p.out = S_[cur]; p.outT = ST_[cur]; p.outT_ident = 1; p.count = 1; p.check = 1;
        int ev = timed ? tm_.begin(0) : -1;
        DL_HIP(launch_nt_step(prec_, cfg_, p, s_));
        tm_.end(ev);
      } else {
        p.X = Yop_; p.Y = S_[prev]; p.add_identity = 0;
        p.out = Tmp_; p.outT = nullptr; p.count = 0; p.check = 1;
        int ev = timed ? tm_.begin(0) : -1;
        DL_HIP(launch_nt_step(prec_, cfg_, p, s_));
        tm_.end(ev);
        p.X = Tmp_; p.Y = Yop_; p.add_identity = 1;
        p.out = S_[cur]; p.outT = nullptr; p.count = 1; p.check = 0;
        if (use_sk_)
          DL_HIP(launch_nt_sym_sk(p, skq_, s_));
        else
          DL_HIP(launch_nt_step(prec_, cfg_, p, s_));
      }
    }
    const int64_t upto = s0_ + cnt - 1;
    s0_ += cnt;
    chunk_ = (mode_ == M_SQUARE && s0_ == 8) ? 4 : std::min(mode_ == M_SG ? chunk_ + chunk_ / 2 : chunk_ * 2, 256);
    return readback(upto);
  }

  // Write the ring and the convergence step to pinned host memory after a
  // chunk (a kernel: a runtime copy left a ~10 us gap before it).  The ring
  // holds the last kRing steps, more than one chunk, so every step of the
  // chunk just run is still present when the host reads it.
  int readback(int64_t upto) {
    DL_HIP(launch_publish(sl_.ring, sl_.h_ring_dev, (int)kSlotWords, s_));
    DL_HIP(hipEventRecord(sl_.ev, s_));
    pending_ = upto;
    return DL_OK;
  }

  // The last iterate computed is R^(computed), in buffer computed % 2.
  int emit() {
    const int64_t last = computed_;
    if (last == 0) {
      DL_HIP(hipMemset2DAsync(R_, (size_t)ldr_, 0, (size_t)n_, (size_t)n_, s_));
    } else {
      const void* src = S_[last & 1];
      const bool in_place = r_is_s0_ && (src == (const void*)R_ || (iters_ >= 2 && last == iters_));
      if (!in_place) DL_HIP(launch_emit(prec_, src, (int)Np_, mode_ == M_PLAIN ? 1 : 0, (int)n_, R_, ldr_, s_));
    }
    done_ = true;
    return DL_OK;
  }

  dl_ctx* c_;
  FixSlot sl_;
  int mode_;
  int64_t n_;
  const uint8_t* A_;
  int64_t lda_;
  uint8_t* R_;
  int64_t ldr_;
  int prec_;
  int32_t max_steps_;
  hipStream_t s_;
  Timer tm_;
  int64_t Np_ = 0;
  int cfg_ = 0;
  NTParams p_{};
  void *Yop_ = nullptr, *S_[2] = {nullptr, nullptr}, *ST_[2] = {nullptr, nullptr}, *Tmp_ = nullptr;
  std::vector<int64_t> ones_ = std::vector<int64_t>(2, 0);
  int64_t iters_ = -1;  // set when the repeat is seen
  int64_t computed_ = 0;
  int64_t s0_ = 2;
  int64_t pending_ = 0;
  int chunk_ = 0;
  bool done_ = false;
  bool r_is_s0_ = false;  // the caller's R is iterate buffer S[0]
  bool use_sk_ = false;   // same generation: S' by the stream-K symmetric product
  SkParams skq_{};
};

// The plain series at small Np as one cooperative launch (k_fix_small): the
// iterates in the slot's workspace, its ring for the model sizes and its
// convergence word for the kernel's status, read back once at the end.  The
// kernel writes R itself.
constexpr long long kFixSmallWaitTicks = 200000000;  // 2 s of s_memrealtime (100 MHz)

int run_plain_whole(dl_ctx* c, uint8_t* ws, int64_t n, const uint8_t* A, int64_t lda, uint8_t* R, int64_t ldr,
                    int prec, int32_t max_steps, int64_t* ones_out, int32_t* steps_out, int32_t* converged_out,
                    hipStream_t s) {
  const int64_t Np = padded_size_for(prec, n);
  const size_t matT = (size_t)mat_bytes(prec, Np);
  FixSmallParams p{};
  p.A = A;
  p.lda = lda;
  p.R = R;
  p.ldr = ldr;
  p.S[0] = ws;
  p.S[1] = ws + matT;
  p.n = (int)n;
  p.Np = (int)Np;
  p.tiles = (int)(Np / 32);
  p.max_steps = (int)std::min<int64_t>(max_steps, Np + 2);
  p.wait_limit = kFixSmallWaitTicks;
  fix_small_place(p, c->fs_words);
  // results straight into the pinned host ring of slot 0 and the word after it
  p.ring_out = c->h_ring_dev;
  p.status_out = (unsigned*)(c->h_ring_dev + kRing);
  volatile unsigned* st = (volatile unsigned*)(c->h_ring + kRing);
  st[0] = ~0u;
  st[1] = 0u;
  const bool clear = c->fs_dirty;
  c->fs_dirty = true;  // until the launch is known to have ended normally
  DL_HIP(launch_fix_small(prec, p, clear, s));
  // The kernel's last store is its status word in pinned host memory, made
  // after every other store of the launch (R, the model sizes, the cleared
  // counters) has completed: the host spins on it and returns as soon as it
  // appears.  A stream synchronisation would add about 14 us (measured) between
  // the kernel's last store and the host's wake-up; later work on the stream
  // stays ordered after the launch anyway.  Every 4096 polls the stream's
  // state is checked, so that a launch that ends without a status (a fault)
  // is reported instead of awaited.
  bool seen = false;
  for (unsigned polls = 1;; ++polls) {
    if (st[0] != ~0u || st[1] != 0u) {
      seen = true;
      break;
    }
    if ((polls & 4095u) == 0 && hipStreamQuery(s) != hipErrorNotReady) break;
  }
  if (!seen) DL_HIP(hipStreamSynchronize(s));
  if (st[1]) return fail(DL_EHIP, "whole-fixpoint kernel: a wait for other workgroups ran past its time limit");
  if (st[0] == ~0u || st[0] > (unsigned)p.max_steps) return fail(DL_EHIP, "whole-fixpoint kernel reported no result");
  c->fs_dirty = false;
  const volatile unsigned long long* ring = c->h_ring;
  const int64_t K = st[0];
  // the first repeat of the whole matrix's model sizes (at K if it converged)
  int64_t k = 1, conv = 0;
  for (; k <= K; ++k) {
    const unsigned long long prev = k == 1 ? 0ull : ring[k - 1];
    if (ring[k] == prev) {
      conv = 1;
      break;
    }
  }
  const int64_t steps = conv ? k : K;
  if (ones_out)
    for (int64_t j = 0; j <= steps; ++j) ones_out[j] = (int64_t)ring[j];
  if (steps_out) *steps_out = (int32_t)steps;
  if (converged_out) *converged_out = (int32_t)conv;
  return DL_OK;
}

// Runs `count` fixpoints of one size, mode and precision on stream s, with
// up to two in flight: while the host reads one's counters back, the device
// runs the other's products.  Per-fixpoint outputs are indexed by g;
// ones_out (model sizes per step) is taken for count == 1 only.
int run_fixpoints(dl_ctx* c, int mode, int count, int64_t n, const uint8_t* const* A, int64_t lda,
                  uint8_t* const* R, int64_t ldr, int prec, int32_t max_steps, int64_t* ones_out,
                  int32_t* steps_out, int32_t* converged_out, hipStream_t s) {
  if (prec < P_I8 || prec > P_FP4) return fail(DL_EINVAL, "unknown precision");
  if (max_steps < 0) return fail(DL_EINVAL, "max_steps < 0");
  if (count <= 0) return DL_OK;
  int rc = set_device(c);
  if (rc) return rc;
  if (n == 0) {
    for (int g = 0; g < count; ++g) {
      if (ones_out && g == 0) {
        ones_out[0] = 0;
        if (max_steps >= 1) ones_out[1] = 0;
      }
      if (steps_out) steps_out[g] = max_steps >= 1 ? 1 : 0;
      if (converged_out) converged_out[g] = max_steps >= 1 ? 1 : 0;
    }
    return DL_OK;
  }
  const int64_t Np = padded_size_for(prec, n);
  size_t need = fix_ws_bytes(prec, Np);
  if (mode == M_SG && sk_supported(prec, pick_config(c, prec, Np), Np)) {
    SkParams q{};
    sk_plan(Np, q);
    need += sk_scratch_bytes(q);  // the stream-K scratch of S' (Fix::start)
  }
  // the plain series takes the whole-fixpoint kernel where it applies unless
  // the caller set another configuration for this size (an entry recorded
  // by dl_tune names the fastest product kernel, which this path does not use)
  const TuneEntry* te = nullptr;
  for (const auto& t : c->tuned)
    if (t.prec == prec && t.np == Np) te = &t;
  const bool forced_other = te && te->cfg != kCfgWholeFixpoint && te->ms == 0.0;
  if (mode == M_PLAIN && max_steps >= 1 && fix_small_supported(prec, Np) && !forced_other) {
    if ((rc = ensure_ws(c, need))) return rc;
    for (int g = 0; g < count; ++g)
      if ((rc = run_plain_whole(c, (uint8_t*)c->ws, n, A[g], lda, R[g], ldr, prec, max_steps,
                                g == 0 ? ones_out : nullptr, steps_out ? steps_out + g : nullptr,
                                converged_out ? converged_out + g : nullptr, s)))
        return rc;
    return DL_OK;
  }
  int nslots = count >= 2 ? kFixSlots : 1;
  if (nslots > 1 && c->budget && need * nslots > c->budget) nslots = 1;  // one at a time within the budget
  if ((rc = ensure_ws(c, need * nslots))) return rc;
  FixSlot slots[kFixSlots];
  for (int i = 0; i < nslots; ++i) {
    if (!c->slot_ev[i]) DL_HIP(hipEventCreateWithFlags(&c->slot_ev[i], hipEventDisableTiming));
    slots[i].ws = (uint8_t*)c->ws + need * i;
    // the slot's ring of model sizes, then its convergence step: one read-back
    slots[i].ring = c->ring + kSlotWords * i;
    slots[i].conv = (int*)(slots[i].ring + kRing);
    slots[i].h_ring = c->h_ring + kSlotWords * i;
    slots[i].h_ring_dev = c->h_ring_dev + kSlotWords * i;
    slots[i].h_conv = (int*)(slots[i].h_ring + kRing);
    slots[i].ev = c->slot_ev[i];
  }
  std::vector<Fix> jobs;
  jobs.reserve(count);
  std::vector<int> inflight;  // indices into jobs, oldest first
  int next = 0;
  auto launch = [&](const FixSlot& sl) -> int {
    const int g = next++;
    jobs.emplace_back(c, sl, mode, n, A[g], lda, R[g], ldr, prec, max_steps, s);
    int r = jobs.back().start();
    if (r) return r;
    if (!jobs.back().done()) inflight.push_back(g);
    return DL_OK;
  };
  for (int i = 0; i < nslots && next < count; ++i)
    if ((rc = launch(slots[i]))) break;
  // a fixpoint that needed no read-back has freed its slot already
  while (!rc && next < count && (int)inflight.size() < nslots) {
    const FixSlot* freed = nullptr;
    for (int i = 0; i < nslots && !freed; ++i) {
      bool busy = false;
      for (int g : inflight) busy = busy || jobs[g].slot().ws == slots[i].ws;
      if (!busy) freed = &slots[i];
    }
    rc = launch(*freed);
  }
  while (!rc && !inflight.empty()) {
    const int g = inflight.front();
    inflight.erase(inflight.begin());
    // poll rather than block: the next chunk is enqueued as soon as the
    // read-back lands (a blocking wait adds the thread's wake-up latency)
    hipError_t e;
    while ((e = hipEventQuery(jobs[g].slot().ev)) == hipErrorNotReady) {
    }
    if (e != hipSuccess) {
      rc = hip_fail(e, "hipEventQuery(read-back)");
      break;
    }
    if ((rc = jobs[g].advance())) break;
    if (!jobs[g].done()) {
      inflight.push_back(g);
    } else if (next < count) {
      // the emit just enqueued is ordered before the next ingest into this slot
      if ((rc = launch(jobs[g].slot()))) break;
    }
  }
  hipError_t e = hipStreamSynchronize(s);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  for (int g = 0; g < count; ++g)
    jobs[g].finish(g == 0 ? ones_out : nullptr, steps_out ? steps_out + g : nullptr,
                   converged_out ? converged_out + g : nullptr);
  if (c->ev_cursor > kMaxPendingEvents) resolve_timing(c);  // bound the event pool
  return DL_OK;
}

}  // namespace

extern "C" {

int dl_create(dl_ctx** out, int device, size_t budget) {
  if (!out) return fail(DL_EINVAL, "ctx out-pointer is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= ndev) return fail(DL_EINVAL, "no such device");
  dl_ctx* c = new (std::nothrow) dl_ctx();
  if (!c) return fail(DL_ENOMEM, "host allocation failed");
  c->device = device;
  c->budget = budget;
  auto cleanup = [&](int st) {
    dl_destroy(c);
    return st;
  };
  if ((e = hipSetDevice(device)) != hipSuccess) return cleanup(hip_fail(e, "hipSetDevice"));
  if ((e = bool_kernels_init()) != hipSuccess) return cleanup(hip_fail(e, "kernel attributes"));
  if ((e = dl::eps_kernels_init()) != hipSuccess) return cleanup(hip_fail(e, "kernel attributes"));
  if ((e = hipMalloc(&c->ring, kFixSlots * kSlotWords * sizeof(unsigned long long))) != hipSuccess)
    return cleanup(hip_fail(e, "hipMalloc(ring)"));
  if ((e = hipMalloc(&c->conv, 64 * sizeof(int))) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc(conv)"));
  c->dscratch = c->conv + 16;
  // coherent: the device's writes of the read-back reach host memory without
  // a cache in between; the slot event after them orders them for the host
  if ((e = hipHostMalloc(&c->h_ring, kFixSlots * kSlotWords * sizeof(unsigned long long),
                         hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess)
    return cleanup(hip_fail(e, "hipHostMalloc(ring)"));
  if ((e = hipHostGetDevicePointer((void**)&c->h_ring_dev, c->h_ring, 0)) != hipSuccess)
    return cleanup(hip_fail(e, "hipHostGetDevicePointer(ring)"));
  if ((e = hipHostMalloc(&c->h_conv, 64 * sizeof(int), hipHostMallocDefault)) != hipSuccess)
    return cleanup(hip_fail(e, "hipHostMalloc(conv)"));
  if ((e = hipMemset(c->ring, 0, kFixSlots * kSlotWords * sizeof(unsigned long long))) != hipSuccess)
    return cleanup(hip_fail(e, "hipMemset(ring)"));
  if ((e = hipMemset(c->conv, 0, 64 * sizeof(int))) != hipSuccess) return cleanup(hip_fail(e, "hipMemset(conv)"));
  {
    const size_t fsb = (size_t)fix_small_words(512) * sizeof(unsigned);
    if ((e = hipMalloc(&c->fs_words, fsb)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc(fixpoint counters)"));
    if ((e = hipMemset(c->fs_words, 0, fsb)) != hipSuccess) return cleanup(hip_fail(e, "hipMemset(fixpoint counters)"));
  }
  if ((e = hipDeviceSynchronize()) != hipSuccess) return cleanup(hip_fail(e, "init sync"));
  *out = c;
  return DL_OK;
}

int dl_destroy(dl_ctx* c) {
  if (!c) return DL_OK;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  if (c->ws) (void)hipFree(c->ws);
  if (c->ring) (void)hipFree(c->ring);
  if (c->conv) (void)hipFree(c->conv);
  if (c->fs_words) (void)hipFree(c->fs_words);
  if (c->h_ring) (void)hipHostFree(c->h_ring);
  if (c->h_conv) (void)hipHostFree(c->h_conv);
  for (auto& ep : c->events) {
    (void)hipEventDestroy(ep.a);
    (void)hipEventDestroy(ep.b);
  }
  for (auto& ev : c->slot_ev)
    if (ev) (void)hipEventDestroy(ev);
  dl::eps_release(&c->eps);
  delete c;
  return DL_OK;
}

int dl_tc_steps(dl_ctx* ctx, int64_t n, const uint8_t* A, int64_t lda, uint8_t* R, int64_t ldr,
                int method, int prec, int32_t max_steps, int64_t* ones, int32_t* steps,
                int32_t* converged, void* stream) {
  int rc = check_common(ctx, n, A, lda, R, ldr);
  if (rc) return rc;
  if (method != DL_TC_PLAIN && method != DL_TC_SQUARE) return fail(DL_EINVAL, "unknown method");
  return run_fixpoints(ctx, method == DL_TC_PLAIN ? M_PLAIN : M_SQUARE, 1, n, &A, lda, &R, ldr, prec, max_steps,
                       ones, steps, converged, (hipStream_t)stream);
}

int dl_tc(dl_ctx* ctx, int64_t n, const uint8_t* A, int64_t lda, uint8_t* R, int64_t ldr, int method,
          int prec, int32_t* iters, void* stream) {
  // plain: iters <= D + 1 <= n + 1; squaring: iters <= 2 + ceil(log2 n)
  int64_t cap = method == DL_TC_SQUARE ? 3 + 64 : n + 2;
  int32_t steps = 0, conv = 0;
  int rc = dl_tc_steps(ctx, n, A, lda, R, ldr, method, prec, (int32_t)std::min<int64_t>(cap, INT_MAX), nullptr,
                       &steps, &conv, stream);
  if (rc) return rc;
  if (!conv) return fail(DL_ENOCONV, "step cap reached before the fixpoint");
  if (iters) *iters = steps;
  return DL_OK;
}

int dl_tc_batch(dl_ctx* ctx, int32_t count, int64_t n, const uint8_t* const* A, int64_t lda, uint8_t* const* R,
                int64_t ldr, int method, int prec, int32_t* iters, void* stream) {
  if (!ctx) return fail(DL_EINVAL, "ctx is NULL");
  if (count < 0) return fail(DL_EINVAL, "count < 0");
  if (count == 0) return DL_OK;
  if (!A || !R || !iters) return fail(DL_EINVAL, "NULL array argument");
  if (method != DL_TC_PLAIN && method != DL_TC_SQUARE) return fail(DL_EINVAL, "unknown method");
  for (int g = 0; g < count; ++g) {
    int rc = check_common(ctx, n, A[g], lda, R[g], ldr);
    if (rc) return rc;
  }
  if (n > 0) {
    const size_t ra = mat_span(n, ldr), aa = mat_span(n, lda);
    for (int g = 0; g < count; ++g)
      for (int h = 0; h < count; ++h) {
        if (h != g && overlaps(R[g], ra, A[h], aa)) return fail(DL_EINVAL, "an output overlaps another input");
        if (h > g && overlaps(R[g], ra, R[h], ra)) return fail(DL_EINVAL, "two outputs overlap");
      }
  }
  // plain: iters <= D + 1 <= n + 1; squaring: iters <= 2 + ceil(log2 n)
  const int64_t cap = method == DL_TC_SQUARE ? 3 + 64 : n + 2;
  std::vector<int32_t> conv(count, 0);
  int rc = run_fixpoints(ctx, method == DL_TC_PLAIN ? M_PLAIN : M_SQUARE, count, n, A, lda, R, ldr, prec,
                         (int32_t)std::min<int64_t>(cap, INT_MAX), nullptr, iters, conv.data(), (hipStream_t)stream);
  if (rc) return rc;
  for (int g = 0; g < count; ++g)
    if (!conv[g]) return fail(DL_ENOCONV, "step cap reached before the fixpoint");
  return DL_OK;
}

int dl_tune(dl_ctx* ctx, int prec, int64_t n, int32_t* cfg_out, double* ms_out, double* cand_ms, void* stream) {
  if (!ctx) return fail(DL_EINVAL, "ctx is NULL");
  if (prec < P_I8 || prec > P_FP4) return fail(DL_EINVAL, "unknown precision");
  if (n <= 0 || n > (1 << 16)) return fail(DL_EINVAL, "n must be in 1 .. 65536");
  int rc = set_device(ctx);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int64_t Np = padded_size_for(prec, n);
  const size_t mat8 = (size_t)Np * Np, matT = (size_t)mat_bytes(prec, Np);
  // [X][Y][out][outT][raw int8]: the operands of one squaring step
  if ((rc = ensure_ws(ctx, fix_ws_bytes(prec, Np) + mat8))) return rc;
  uint8_t* base = (uint8_t*)ctx->ws;
  uint8_t* op[4];
  for (int i = 0; i < 4; ++i) op[i] = base + i * matT;
  uint8_t* raw = base + 4 * matT;
  DL_HIP(launch_hash_bool(raw, Np, (int)n, (int)Np, 0x5eedu, s));
  DL_HIP(launch_ingest(prec, raw, Np, (int)n, (int)Np, nullptr, nullptr, op[0], op[1], 2, nullptr, s));
  NTParams p{};  // a squaring step, as the fixpoint driver launches it
  p.X = op[0];
  p.Y = op[1];
  p.out = op[2];
  p.outT = op[3];
  p.outT_ident = 1;
  p.ld = Np;
  p.Np = (int)Np;
  p.n_valid = (int)n;
  p.ones = ctx->ring;
  p.conv = nullptr;  // never returns early
  p.step = 2;
  p.count = 1;
  hipEvent_t ea = nullptr, eb = nullptr;
  DL_HIP(hipEventCreate(&ea));
  if (hipEventCreate(&eb) != hipSuccess) {
    (void)hipEventDestroy(ea);
    return fail(DL_EHIP, "hipEventCreate");
  }
  // average time of `reps` launches of configuration cfg
  auto timed = [&](int cfg, int reps, double* ms) -> hipError_t {
    hipError_t e = hipEventRecord(ea, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_nt_step(prec, cfg, p, s);
    if (e == hipSuccess) e = hipEventRecord(eb, s);
    if (e == hipSuccess) e = hipEventSynchronize(eb);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, ea, eb);
    *ms = (double)t / reps;
    return e;
  };
  // Candidates that apply; each is warmed up, then timed in kRounds rounds
  // that visit the candidates in turn (so slow drifts of the clock affect
  // all of them alike), about 4 ms of launches per candidate and round; a
  // candidate's time is its median over the rounds.
  constexpr int kRounds = 5;
  std::vector<int> cands;
  std::vector<int> reps;
  std::vector<std::vector<double>> samples;
  hipError_t e = hipSuccess;
  auto set_tiles = [&](int cfg) {
    const TileCfg tc = nt_config(prec, cfg);
    p.tiles_m = (int)(Np / tc.bm);
    p.tiles_n = (int)(Np / tc.bn);
  };
  for (int cfg = 0; cfg < nt_config_count(prec) && e == hipSuccess; ++cfg) {
    if (cand_ms) cand_ms[cfg] = -1.0;
    if (!nt_config_valid(prec, cfg, Np)) continue;
    set_tiles(cfg);
    double first = 0.0;
    if ((e = timed(cfg, 1, &first)) != hipSuccess) break;  // warm-up (code load, clocks)
    if ((e = timed(cfg, 1, &first)) != hipSuccess) break;
    cands.push_back(cfg);
    reps.push_back((int)std::min(40.0, std::max(2.0, 4.0 / std::max(first, 1e-3))));
    samples.emplace_back();
  }
  for (int round = 0; round < kRounds && e == hipSuccess; ++round)
    for (size_t i = 0; i < cands.size() && e == hipSuccess; ++i) {
      set_tiles(cands[i]);
      double ms = 0.0;
      if ((e = timed(cands[i], reps[i], &ms)) == hipSuccess) samples[i].push_back(ms);
    }
  (void)hipEventDestroy(ea);
  (void)hipEventDestroy(eb);
  if (e != hipSuccess) return hip_fail(e, "autotune launches");
  int best = -1;
  double best_ms = 0.0, cfg_ms[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (size_t i = 0; i < cands.size(); ++i) {
    std::vector<double>& v = samples[i];
    std::sort(v.begin(), v.end());
    const double ms = v[v.size() / 2];
    cfg_ms[cands[i]] = ms;
    if (cand_ms) cand_ms[cands[i]] = ms;
    if (best < 0 || ms < best_ms) {
      best = cands[i];
      best_ms = ms;
    }
  }
  // keep the size rule's choice unless another configuration beats it by
  // more than 5% (run-to-run noise would otherwise flip near-ties)
  const int def = choose_nt_config(prec, Np);
  if (def != best && cfg_ms[def] > 0.0 && cfg_ms[def] <= 1.05 * best_ms) {
    best = def;
    best_ms = cfg_ms[def];
  }
  bool found = false;
  for (auto& t : ctx->tuned)
    if (t.prec == prec && t.np == Np) {
      t.cfg = best;
      t.ms = best_ms;
      found = true;
    }
  if (!found) ctx->tuned.push_back({prec, Np, best, best_ms});
  if (cfg_out) *cfg_out = best;
  if (ms_out) *ms_out = best_ms;
  return DL_OK;
}

int dl_tune_set(dl_ctx* ctx, int prec, int64_t n, int32_t cfg) {
  if (!ctx) return fail(DL_EINVAL, "ctx is NULL");
  if (prec < P_I8 || prec > P_FP4) return fail(DL_EINVAL, "unknown precision");
  if (n <= 0 || n > (1 << 16)) return fail(DL_EINVAL, "n must be in 1 .. 65536");
  const int64_t Np = padded_size_for(prec, n);
  if (cfg < -1 || (cfg >= 0 && !nt_config_valid(prec, cfg, Np)))
    return fail(DL_EINVAL, "no such tile configuration for this precision and size");
  for (size_t i = 0; i < ctx->tuned.size(); ++i)
    if (ctx->tuned[i].prec == prec && ctx->tuned[i].np == Np) {
      if (cfg < 0) {
        ctx->tuned.erase(ctx->tuned.begin() + i);
      } else {
        ctx->tuned[i].cfg = cfg;
        ctx->tuned[i].ms = 0.0;
      }
      return DL_OK;
    }
  if (cfg >= 0) ctx->tuned.push_back({prec, Np, cfg, 0.0});
  return DL_OK;
}

int dl_tune_get(dl_ctx* ctx, int32_t* prec, int64_t* np, int32_t* cfg, double* ms, int32_t cap, int32_t* count) {
  if (!ctx || !count || cap < 0) return fail(DL_EINVAL, "bad arguments");
  const int32_t k = (int32_t)std::min<size_t>((size_t)cap, ctx->tuned.size());
  for (int32_t i = 0; i < k; ++i) {
    const TuneEntry& t = ctx->tuned[i];
    if (prec) prec[i] = t.prec;
    if (np) np[i] = t.np;
    if (cfg) cfg[i] = t.cfg;
    if (ms) ms[i] = t.ms;
  }
  *count = (int32_t)ctx->tuned.size();
  return DL_OK;
}

int dl_sg_steps(dl_ctx* ctx, int64_t n, const uint8_t* P, int64_t ldp, uint8_t* S, int64_t lds, int prec,
                int32_t max_steps, int64_t* ones, int32_t* steps, int32_t* converged, void* stream) {
  int rc = check_common(ctx, n, P, ldp, S, lds);
  if (rc) return rc;
  return run_fixpoints(ctx, M_SG, 1, n, &P, ldp, &S, lds, prec, max_steps, ones, steps, converged,
                      (hipStream_t)stream);
}

int dl_sg(dl_ctx* ctx, int64_t n, const uint8_t* P, int64_t ldp, uint8_t* S, int64_t lds, int prec,
          int32_t* iters, void* stream) {
  // a new pair needs a pair of equal-length walks to a common constant: at
  // most n^2 rounds after the diagonal
  const int64_t cap = std::min<int64_t>(n * n + 2, INT_MAX);
  int32_t steps = 0, conv = 0;
  int rc = dl_sg_steps(ctx, n, P, ldp, S, lds, prec, (int32_t)cap, nullptr, &steps, &conv, stream);
  if (rc) return rc;
  if (!conv) return fail(DL_ENOCONV, "step cap reached before the fixpoint");
  if (iters) *iters = steps;
  return DL_OK;
}

int dl_eps_bound(dl_ctx* ctx, int64_t n, const uint8_t* A, int64_t lda, double* eps_max, void* stream) {
  if (!ctx || !eps_max) return fail(DL_EINVAL, "NULL argument");
  if (n < 0 || (n > 0 && (!A || lda < n))) return fail(DL_EINVAL, "bad matrix");
  int rc = set_device(ctx);
  if (rc) return rc;
  if (n == 0) {
    *eps_max = 1.0;
    return DL_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  DL_HIP(hipMemsetAsync(ctx->dscratch, 0, sizeof(int), s));
  DL_HIP(launch_row_max(A, lda, (int)n, ctx->dscratch, s));
  DL_HIP(hipMemcpyAsync(ctx->h_conv + 1, ctx->dscratch, sizeof(int), hipMemcpyDeviceToHost, s));
  DL_HIP(hipStreamSynchronize(s));
  *eps_max = 1.0 / (1.0 + (double)ctx->h_conv[1]);
  return DL_OK;
}

int dl_solve_eps(dl_ctx* ctx, int64_t n, const uint8_t* A, int64_t lda, double eps, uint8_t* R, int64_t ldr,
                 double* X, int64_t ldx, int32_t* iters, int32_t* underflow, void* stream) {
  int rc = check_common(ctx, n, A, lda, R, ldr);
  if (rc) return rc;
  if (X && n > 0) {
    if (ldx < n) return fail(DL_EINVAL, "ldx < n");
    if (overlaps(X, mat_span(n, ldx) * sizeof(double), A, mat_span(n, lda)) ||
        overlaps(X, mat_span(n, ldx) * sizeof(double), R, mat_span(n, ldr)))
      return fail(DL_EINVAL, "X overlaps another matrix");
  }
  if (!(eps > 0.0)) return fail(DL_EINVAL, "eps must be positive");
  if (iters) *iters = 0;
  if (underflow) *underflow = 0;
  if (n == 0) return DL_OK;
  double bound = 0.0;
  if ((rc = dl_eps_bound(ctx, n, A, lda, &bound, stream))) return rc;
  if (eps > bound) {
    char buf[160];
    snprintf(buf, sizeof buf, "eps = %.17g exceeds 1/(1+||A||_inf) = %.17g (Lemma 1)", eps, bound);
    return fail(DL_EINVAL, buf);
  }
  hipStream_t s = (hipStream_t)stream;
  std::string err;
  double tmsum = 0.0;
  int64_t tcount = 0;
  double minpos = INFINITY;
  hipError_t e = dl::eps_solve(&ctx->eps, ctx->budget, n, A, lda, A, lda, eps, R, ldr, X, ldx, s, ctx->timing,
                               &tmsum, &tcount, &minpos, &err);
  if (e == hipErrorOutOfMemory) return fail(DL_ENOMEM, err);
  if (e != hipSuccess) return fail(DL_EHIP, err + ": " + hipGetErrorString(e));
  ctx->ms[1] += tmsum;
  ctx->launches[1] += tcount;
  // X = eps A + eps A X, so along a shortest path i -> v -> ... -> j the
  // true entries X_vj, X_ij shrink by at most a factor eps per edge, from
  // X_.j >= eps at the last edge.  A true entry below the smallest normal
  // double therefore implies one in [DBL_MIN, DBL_MIN / eps), which the
  // elimination computes to full relative accuracy; if the smallest positive
  // entry computed is at least twice that, no true entry is that small and
  // none was lost.
  if (underflow) *underflow = minpos < 2.0 * DBL_MIN / eps ? 1 : 0;
  return DL_OK;
}

int dl_sg_eps(dl_ctx* ctx, int64_t n, const uint8_t* P, int64_t ldp, double eps, uint8_t* S, int64_t lds,
              double* X, int64_t ldx, int32_t* doublings, void* stream) {
  int rc = check_common(ctx, n, P, ldp, S, lds);
  if (rc) return rc;
  if (X && n > 0) {
    if (ldx < n) return fail(DL_EINVAL, "ldx < n");
    if (overlaps(X, mat_span(n, ldx) * sizeof(double), P, mat_span(n, ldp)) ||
        overlaps(X, mat_span(n, ldx) * sizeof(double), S, mat_span(n, lds)))
      return fail(DL_EINVAL, "X overlaps another matrix");
  }
  if (!(eps > 0.0)) return fail(DL_EINVAL, "eps must be positive");
  if (doublings) *doublings = 0;
  if (n == 0) return DL_OK;
  double bound1 = 0.0;
  if ((rc = dl_eps_bound(ctx, n, P, ldp, &bound1, stream))) return rc;
  const double d = std::round(1.0 / bound1 - 1.0);  // max row sum of P (an integer)
  const double bound = 1.0 / (1.0 + d * d);
  if (eps > bound * (1.0 + 1e-15)) {
    char buf[160];
    snprintf(buf, sizeof buf, "eps = %.17g exceeds 1/(1+||P||_inf^2) = %.17g", eps, bound);
    return fail(DL_EINVAL, buf);
  }
  std::string err;
  int32_t dbl = 0;
  int64_t pos = 0;
  hipError_t e = dl::sg_eps_solve(&ctx->eps, ctx->budget, n, P, ldp, eps, S, lds, X, ldx, 64, (hipStream_t)stream,
                                  &dbl, &pos, (unsigned long long*)(ctx->dscratch + 8), ctx->h_ring, &err);
  if (e == hipErrorOutOfMemory) return fail(DL_ENOMEM, err);
  if (e == hipErrorNotReady) return fail(DL_ENOCONV, "doubling cap reached");
  if (e != hipSuccess) return fail(DL_EHIP, err + ": " + hipGetErrorString(e));
  if (doublings) *doublings = dbl;
  return DL_OK;
}

int dl_solve_linear(dl_ctx* ctx, int64_t n, const uint8_t* B, int64_t ldb, const uint8_t* C, int64_t ldc,
                    double eps, uint8_t* R, int64_t ldr, double* X, int64_t ldx, void* stream) {
  int rc = check_common(ctx, n, B, ldb, R, ldr);
  if (rc) return rc;
  if ((rc = check_common(ctx, n, C, ldc, R, ldr))) return rc;
  if (X && n > 0) {
    if (ldx < n) return fail(DL_EINVAL, "ldx < n");
    const size_t xs = mat_span(n, ldx) * sizeof(double);
    if (overlaps(X, xs, B, mat_span(n, ldb)) || overlaps(X, xs, C, mat_span(n, ldc)) ||
        overlaps(X, xs, R, mat_span(n, ldr)))
      return fail(DL_EINVAL, "X overlaps another matrix");
  }
  if (!(eps > 0.0)) return fail(DL_EINVAL, "eps must be positive");
  if (n == 0) return DL_OK;
  double bound = 0.0;
  if ((rc = dl_eps_bound(ctx, n, B, ldb, &bound, stream))) return rc;
  if (eps > bound) {
    char buf[160];
    snprintf(buf, sizeof buf, "eps = %.17g exceeds 1/(1+||B||_inf) = %.17g", eps, bound);
    return fail(DL_EINVAL, buf);
  }
  std::string err;
  double tmsum = 0.0;
  int64_t tcount = 0;
  hipError_t e = dl::eps_solve(&ctx->eps, ctx->budget, n, B, ldb, C, ldc, eps, R, ldr, X, ldx, (hipStream_t)stream,
                               false, &tmsum, &tcount, nullptr, &err);
  if (e == hipErrorOutOfMemory) return fail(DL_ENOMEM, err);
  if (e != hipSuccess) return fail(DL_EHIP, err + ": " + hipGetErrorString(e));
  return DL_OK;
}

int dl_solve_two_sided(dl_ctx* ctx, int64_t n, const uint8_t* Q, int64_t ldq, const uint8_t* B, int64_t ldb,
                       const uint8_t* C, int64_t ldc, double eps, uint8_t* R, int64_t ldr, double* X, int64_t ldx,
                       int32_t* doublings, void* stream) {
  int rc;
  if ((rc = check_common(ctx, n, Q, ldq, R, ldr))) return rc;
  if ((rc = check_common(ctx, n, B, ldb, R, ldr))) return rc;
  if ((rc = check_common(ctx, n, C, ldc, R, ldr))) return rc;
  if (X && n > 0) {
    if (ldx < n) return fail(DL_EINVAL, "ldx < n");
    const size_t xs = mat_span(n, ldx) * sizeof(double);
    if (overlaps(X, xs, Q, mat_span(n, ldq)) || overlaps(X, xs, B, mat_span(n, ldb)) ||
        overlaps(X, xs, C, mat_span(n, ldc)) || overlaps(X, xs, R, mat_span(n, ldr)))
      return fail(DL_EINVAL, "X overlaps another matrix");
  }
  if (!(eps > 0.0)) return fail(DL_EINVAL, "eps must be positive");
  if (doublings) *doublings = 0;
  if (n == 0) return DL_OK;
  if ((rc = set_device(ctx))) return rc;
  hipStream_t s = (hipStream_t)stream;
  // ||B||_inf (max row sum) and ||C||_1 (max column sum)
  DL_HIP(hipMemsetAsync(ctx->dscratch, 0, 2 * sizeof(int), s));
  DL_HIP(launch_row_max(B, ldb, (int)n, ctx->dscratch, s));
  DL_HIP(launch_col_max(C, ldc, (int)n, ctx->dscratch + 1, s));
  DL_HIP(hipMemcpyAsync(ctx->h_conv + 1, ctx->dscratch, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  DL_HIP(hipStreamSynchronize(s));
  const double bound = 1.0 / (1.0 + (double)ctx->h_conv[1] * (double)ctx->h_conv[2]);
  if (eps > bound * (1.0 + 1e-15)) {
    char buf[160];
    snprintf(buf, sizeof buf, "eps = %.17g exceeds 1/(1+||C||_1 ||B||_inf) = %.17g", eps, bound);
    return fail(DL_EINVAL, buf);
  }
  std::string err;
  int32_t dbl = 0;
  hipError_t e = dl::two_sided_solve(&ctx->eps, ctx->budget, n, Q, ldq, B, ldb, C, ldc, eps, R, ldr, X, ldx, nullptr, 0,
                                     nullptr, 64, s, &dbl, (unsigned long long*)(ctx->dscratch + 8), ctx->h_ring,
                                     &err);
  if (e == hipErrorOutOfMemory) return fail(DL_ENOMEM, err);
  if (e == hipErrorNotReady) return fail(DL_ENOCONV, "doubling cap reached");
  if (e != hipSuccess) return fail(DL_EHIP, err + ": " + hipGetErrorString(e));
  if (doublings) *doublings = dbl;
  return DL_OK;
}

int dl_measure_peak(dl_ctx* ctx, int kind, double* ops_per_s, void* stream) {
  if (!ctx || !ops_per_s) return fail(DL_EINVAL, "NULL argument");
  if (kind < 0 || kind > 8) return fail(DL_EINVAL, "unknown kind");
  int rc = set_device(ctx);
  if (rc) return rc;
  if (kind == 7 && (rc = ensure_ws(ctx, 1 << 20))) return rc;
  DL_HIP(measure_peak(kind, (int*)ctx->ring, ops_per_s, (hipStream_t)stream, (const uint8_t*)ctx->ws));
  return DL_OK;
}

int dl_set_timing(dl_ctx* ctx, int enable) {
  if (!ctx) return fail(DL_EINVAL, "ctx is NULL");
  if (enable) {
    // event pairs made here rather than on the first launches they bracket
    // (creating events between launches delays the launches behind them)
    int rc = set_device(ctx);
    if (rc) return rc;
    constexpr size_t kInitialPairs = 256;
    while (ctx->events.size() < kInitialPairs) {
      EventPair ep;
      DL_HIP(hipEventCreate(&ep.a));
      hipError_t e = hipEventCreate(&ep.b);
      if (e != hipSuccess) {
        (void)hipEventDestroy(ep.a);
        return hip_fail(e, "hipEventCreate");
      }
      ctx->events.push_back(ep);
    }
  }
  ctx->timing = enable != 0;
  return DL_OK;
}

int dl_kernel_stats(dl_ctx* ctx, int cls, int64_t* launches, double* total_ms, int reset) {
  if (!ctx || cls < 0 || cls > 2) return fail(DL_EINVAL, "bad argument");
  int rc = set_device(ctx);
  if (rc) return rc;
  resolve_timing(ctx);
  if (launches) *launches = ctx->launches[cls];
  if (total_ms) *total_ms = ctx->ms[cls];
  if (reset) {
    ctx->launches[cls] = 0;
    ctx->ms[cls] = 0.0;
  }
  return DL_OK;
}

int64_t dl_padded_size(int64_t n, int kind, int prec) {
  if (kind == 2) return dl::eps_padded_size(n);
  return padded_size_for(prec, n);
}

const char* dl_status_str(int status) {
  switch (status) {
    case DL_OK: return "DL_OK";
    case DL_EINVAL: return "DL_EINVAL: invalid argument";
    case DL_ENOMEM: return "DL_ENOMEM: out of memory or over budget";
    case DL_EHIP: return "DL_EHIP: HIP runtime error";
    case DL_ENOCONV: return "DL_ENOCONV: step cap reached";
    case DL_EUNSUPPORTED: return "DL_EUNSUPPORTED: unsupported method/precision";
    case DL_EAGAIN: return "DL_EAGAIN: no free batch slot or pool memory";
    default: return "unknown status";
  }
}

const char* dl_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
