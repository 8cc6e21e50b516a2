// ctx.h -- the library context behind the opaque dl_ctx of include/dl.h
// (internal to the library's sources).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "eps_solve.h"

struct EventPair {
  hipEvent_t a, b;
};

struct dl_ctx {
  int device = 0;
  size_t budget = 0;
  void* ws = nullptr;  // main workspace
  size_t ws_size = 0;
  unsigned long long* ring = nullptr;  // device ring of model sizes (kRing slots)
  int* conv = nullptr;                 // device convergence step
  int* dscratch = nullptr;             // small device scratch (row max, ...)
  unsigned long long* h_ring = nullptr;  // pinned host mirror of the ring
  int* h_conv = nullptr;                 // pinned: conv step, scratch ints
  bool timing = false;
  int64_t launches[3] = {0, 0, 0};
  double ms[3] = {0, 0, 0};
  std::vector<EventPair> events;
  dl::EpsWorkspace eps;  // workspace of the epsilon solve
};

namespace dl {
void set_last_error(const std::string& m);
}  // namespace dl
