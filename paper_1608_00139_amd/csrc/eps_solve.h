// eps_solve.h -- fp64 solve of the purely linear epsilon form.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace dl {

struct EpsWorkspace {
  void* buf = nullptr;
  size_t size = 0;
};

void eps_free(EpsWorkspace* ws);
int64_t eps_padded_size(int64_t n);

// Solves (I - eps A) X = eps A for X (fp64) and writes R = [X > 0] (n x n,
// ldr) and, if X_out is not null, X (n x n, ldx).  `budget_left` caps the
// workspace (0 = no cap).  With timing on, the trailing-update launches are
// bracketed by events and their count and total time are returned.
hipError_t eps_solve(EpsWorkspace* ws, size_t budget_left, int64_t n, const uint8_t* A, int64_t lda,
                     double eps, uint8_t* R, int64_t ldr, double* X_out, int64_t ldx, hipStream_t s,
                     bool timing, double* trailing_ms, int64_t* trailing_launches, std::string* err);

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

}  // namespace dl
