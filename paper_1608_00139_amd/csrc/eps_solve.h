// eps_solve.h -- fp64 solve of the purely linear epsilon form.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace dl {

struct EpsWorkspace {
  void* buf = nullptr;
  size_t size = 0;
  hipStream_t side = nullptr;  // look-ahead stream of the elimination (default priority)
  hipStream_t work = nullptr;  // the elimination's main stream (default priority)
  bool masked = false;         // work and side run on disjoint compute units
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};

// eps_free releases the buffer; eps_release also the stream and events.
void eps_free(EpsWorkspace* ws);
void eps_release(EpsWorkspace* ws);
// Kernel attributes (once per device, at context creation).
hipError_t eps_kernels_init();
int64_t eps_padded_size(int64_t n);

// Solves (I - eps B) X = eps C for X (fp64; B, C caller 0/1 bytes, nonzero =
// true) and writes R = [X > 0] (n x n, ldr) and, if X_out is not null, X
// (n x n, ldx).  B = C = A is the closure form.  `budget_left` caps the
// workspace (0 = no cap).  With timing on, the trailing-update launches are
// bracketed by events and their count and total time are returned.
// min_positive (host, may be null) receives the smallest positive entry of X
// (+inf when X has none).
hipError_t eps_solve(EpsWorkspace* ws, size_t budget_left, int64_t n, const uint8_t* B, int64_t ldb,
                     const uint8_t* C, int64_t ldc, double eps, uint8_t* R, int64_t ldr, double* X_out,
                     int64_t ldx, hipStream_t s, bool timing, double* trailing_ms, int64_t* trailing_launches,
                     double* min_positive, std::string* err);

// One layer of tail-recursive heads h = 0 .. M-1,
//   X_h = eps_h (A_h + sum_j B[h][j] X_j),
// solved as one stacked linear system; all matrices are int8 0/1 Np x Np
// (row-major, zero padded, null = zero).  R[h] receives [X_h > 0] and, if
// cnt is set, cnt[h] += its number of ones (cnt must be cleared first).
constexpr int kMaxStack = 8;
struct StackDesc {
  int M = 0;
  int Np = 0;
  const int8_t* B[kMaxStack][kMaxStack] = {};
  const int8_t* A[kMaxStack] = {};
  double eps[kMaxStack] = {};
  int8_t* R[kMaxStack] = {};
  int64_t ldr = 0;  // row stride of the R[h] (0: Np)
  unsigned long long* cnt = nullptr;
};
hipError_t stacked_solve(EpsWorkspace* ws, size_t budget_left, const StackDesc& d, hipStream_t s, std::string* err);

// Same-generation epsilon form X = eps (I + P X P^T) by Smith's doubling in
// fp64; writes S = [X > 0] and optionally X.  Stops when a doubling adds no
// positive entry and, if X_out is given, also changes no value.  *doublings
// receives the number of doublings run, the last one confirming the fixpoint;
// hipErrorNotReady if max_doublings ran out first.  d_counter / h_counter: two
// device and two pinned host 64-bit words.
hipError_t sg_eps_solve(EpsWorkspace* ws, size_t budget_left, int64_t n, const uint8_t* P, int64_t ldp, double eps,
                        uint8_t* S, int64_t lds, double* X_out, int64_t ldx, int max_doublings, hipStream_t s,
                        int32_t* doublings, int64_t* positives, unsigned long long* d_counter,
                        unsigned long long* h_counter, std::string* err);

// Two-sided equation X = eps (Q + B X C) (Q, B, C 0/1 bytes with leading
// dimensions; n x n) by the same doubling with B and C each scaled by
// sqrt(eps).  Outputs (any may be null): R = [X > 0] as caller bytes (ldr), X
// (ldx), and R8 = [X > 0] as int8 rows of stride ld8 >= n (rows and columns
// from n up to the solver's padded size are written as zeros; the caller
// clears anything beyond) with its ones added to *r8_count.
hipError_t two_sided_solve(EpsWorkspace* ws, size_t budget_left, int64_t n, const uint8_t* Q, int64_t ldq,
                           const uint8_t* B, int64_t ldb, const uint8_t* C, int64_t ldc, double eps, uint8_t* R,
                           int64_t ldr, double* X_out, int64_t ldx, int8_t* R8, int64_t ld8,
                           unsigned long long* r8_count, int max_doublings, hipStream_t s, int32_t* doublings, unsigned long long* d_counter,
                           unsigned long long* h_counter, std::string* err);

}  // namespace dl
