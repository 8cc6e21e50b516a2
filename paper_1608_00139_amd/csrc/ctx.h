// ctx.h -- the library context behind the opaque dl_ctx of include/dl.h
// (internal to the library's sources).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "eps_solve.h"

// Fixpoints a batched call keeps in flight (each with its own workspace,
// counters and read-back event).
constexpr int kFixSlots = 2;

struct EventPair {
  hipEvent_t a, b;
};

struct dl_ctx {
  int device = 0;
  size_t budget = 0;
  void* ws = nullptr;  // main workspace
  size_t ws_size = 0;
  unsigned long long* ring = nullptr;  // device rings of model sizes (kRing per fixpoint slot)
  int* conv = nullptr;                 // device convergence steps (conv[4 i] for slot i)
  int* dscratch = nullptr;             // small device scratch (row max, ...)
  unsigned long long* h_ring = nullptr;  // pinned host mirror of the rings
  int* h_conv = nullptr;                 // pinned: conv steps (h_conv[4 i]), scratch ints
  hipEvent_t slot_ev[kFixSlots] = {nullptr, nullptr};  // read-back events of the fixpoint slots
  bool timing = false;
  int64_t launches[3] = {0, 0, 0};
  double ms[3] = {0, 0, 0};
  std::vector<EventPair> events;
  dl::EpsWorkspace eps;  // workspace of the epsilon solve
};

namespace dl {
void set_last_error(const std::string& m);
}  // namespace dl
