// noalloc.cpp -- dl_tc_noalloc: the plain closure fixpoint for small relations
// with every device buffer it needs in a file-scope device array, for callers
// that cannot allocate device memory.
//
// The array `scratch` below is a device symbol: in host code its name is only
// a stand-in, so the first call on each device looks up its device address
// (hipGetSymbolAddress, with that device current) and every later use goes
// through that address.  Each device holds its own copy of the array for the
// life of the process.  Calls on one device share the copy: they must not
// overlap (they race), and each call leaves the counters in it zeroed for the
// next (after an abnormal end the next call on that device clears them
// first).
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>

#include "../../include/dl.h"
#include "common.h"

namespace dl {
void set_last_error(const std::string& m);
}

using namespace dl;

namespace {

constexpr int64_t kNoAllocMaxNp = 512;  // the one-launch kernel's limit
// Layout of the array: two iterates of the largest size (fp32, Np = 512),
// the kernel's counters, then its outputs: status (2 words) and the ring of
// model sizes (Np + 3 entries).
constexpr size_t kIterBytes = (size_t)kNoAllocMaxNp * kNoAllocMaxNp * 4;
constexpr size_t kCountersOff = 2 * kIterBytes;
constexpr size_t kCountersBytes = ((size_t)(3 * (kNoAllocMaxNp / 32) * (kNoAllocMaxNp + 3) + kNoAllocMaxNp / 32 + 2) *
                                       sizeof(unsigned) + 255) / 256 * 256;
constexpr size_t kOutOff = kCountersOff + kCountersBytes;
constexpr size_t kOutWords = 1 + (kNoAllocMaxNp + 3);  // status (two 32-bit words), then the ring
constexpr size_t kScratchBytes = kOutOff + kOutWords * 8;
constexpr int kMaxDevices = 64;
constexpr long long kWaitTicks = 200000000;  // 2 s of s_memrealtime (100 MHz)

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
bool g_dirty[kMaxDevices] = {};

int fail(int status, const std::string& msg) {
  set_last_error(msg);
  return status;
}

int hip_fail(hipError_t e, const char* what) {
  set_last_error(std::string(what) + ": " + hipGetErrorString(e));
  return DL_EHIP;
}

// The device address of this device's copy of `scratch` (looked up once per
// device, with the device current) and its dirty flag.
int scratch_of(int dev, void** ptr) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_ptr[dev] = p;
    g_dirty[dev] = true;  // clear once before the first launch
  }
  *ptr = g_ptr[dev];
  return DL_OK;
}

bool overlaps(const void* a, size_t alen, const void* b, size_t blen) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + blen && y < x + alen;
}

}  // namespace

extern "C" int dl_tc_noalloc(int64_t n, const uint8_t* A, int64_t lda, uint8_t* R, int64_t ldr, int prec,
                             int32_t* iters, void* stream) {
  if (n < 0) return fail(DL_EINVAL, "n < 0");
  if (prec < P_I8 || prec > P_FP4) return fail(DL_EINVAL, "unknown precision");
  if (n == 0) {
    if (iters) *iters = 1;
    return DL_OK;
  }
  const int64_t Np = padded_size_for(prec, n);
  if (Np > kNoAllocMaxNp || !fix_small_supported(prec, Np))
    return fail(DL_EINVAL, "n = " + std::to_string(n) + " exceeds the no-allocation limit (" +
                               std::to_string(kNoAllocMaxNp) + " constants)");
  if (!A || !R) return fail(DL_EINVAL, "NULL matrix pointer");
  if (lda < n || ldr < n) return fail(DL_EINVAL, "leading dimension smaller than n");
  if (overlaps(A, (size_t)((n - 1) * lda + n), R, (size_t)((n - 1) * ldr + n)))
    return fail(DL_EINVAL, "the output overlaps the input");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(DL_EINVAL, "device index beyond the supported range");
  void* base = nullptr;
  int rc = scratch_of(dev, &base);
  if (rc) return rc;
  uint8_t* sc = (uint8_t*)base;
  hipStream_t s = (hipStream_t)stream;

  FixSmallParams p{};
  p.A = A;
  p.lda = lda;
  p.R = R;
  p.ldr = ldr;
  p.S[0] = sc;
  p.S[1] = sc + kIterBytes;
  p.n = (int)n;
  p.Np = (int)Np;
  p.tiles = (int)(Np / 32);
  p.max_steps = (int)(Np + 2);  // the plain series repeats by step n + 1
  p.wait_limit = kWaitTicks;
  fix_small_place(p, (unsigned*)(sc + kCountersOff));
  p.status_out = (unsigned*)(sc + kOutOff);
  p.ring_out = (unsigned long long*)(sc + kOutOff + 8);
  bool clear;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    clear = g_dirty[dev];
    g_dirty[dev] = true;  // until this launch is known to have ended normally
  }
  if ((e = launch_fix_small(prec, p, clear, s)) != hipSuccess) return hip_fail(e, "whole-fixpoint launch");
  unsigned long long out[kOutWords];
  const size_t out_bytes = 8 * (size_t)(1 + Np + 3);
  if ((e = hipMemcpyAsync(out, sc + kOutOff, out_bytes, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(e, "read-back of the model sizes");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  unsigned status[2];
  memcpy(status, out, sizeof status);
  if (status[1]) return fail(DL_EHIP, "whole-fixpoint kernel: a wait for other workgroups ran past its time limit");
  const int64_t K = status[0];
  if (K < 1 || K > p.max_steps) return fail(DL_EHIP, "whole-fixpoint kernel reported no result");
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_dirty[dev] = false;
  }
  const unsigned long long* ring = out + 1;
  for (int64_t k = 1; k <= K; ++k) {
    const unsigned long long prev = k == 1 ? 0ull : ring[k - 1];
    if (ring[k] == prev) {
      if (iters) *iters = (int32_t)k;
      return DL_OK;
    }
  }
  return fail(DL_ENOCONV, "step cap reached before the fixpoint");
}
