// ctx.h -- the library context behind the opaque dl_ctx of include/dl.h
// (internal to the library's sources).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "common.h"
#include "eps_solve.h"

// Fixpoints a batched call keeps in flight (each with its own workspace,
// counters and read-back event).
constexpr int kFixSlots = 2;
constexpr size_t kSlotWords = (size_t)dl::kRing + 1;  // a slot's ring and its convergence step

struct EventPair {
  hipEvent_t a, b;
};

// A tile configuration chosen for (precision, padded size) by the autotuner
// or set by the caller; ms is the measured time of one product (0 if set).
struct TuneEntry {
  int prec;
  int64_t np;
  int cfg;
  double ms;
};

struct dl_ctx {
  int device = 0;
  size_t budget = 0;
  void* ws = nullptr;  // main workspace
  size_t ws_size = 0;
  unsigned long long* ring = nullptr;  // per fixpoint slot: kRing model sizes, then the slot's
                                       // convergence step (an int in one more word)
  int* conv = nullptr;                 // device scratch ints (eps bounds, solver flags)
  int* dscratch = nullptr;             // small device scratch (row max, ...)
  unsigned long long* h_ring = nullptr;  // pinned (coherent) host mirror of the slots' rings and steps
  unsigned long long* h_ring_dev = nullptr;  // its device mapping, written by k_publish
  int* h_conv = nullptr;                 // pinned scratch ints
  hipEvent_t slot_ev[kFixSlots] = {nullptr, nullptr};  // read-back events of the fixpoint slots
  bool timing = false;
  int64_t launches[3] = {0, 0, 0};
  double ms[3] = {0, 0, 0};
  std::vector<EventPair> events;    // pool of timing event pairs
  size_t ev_cursor = 0;             // pairs [0, ev_cursor) hold launches not yet resolved
  std::vector<std::pair<int, int>> pending;  // (class, pair index) to add to ms / launches
  dl::EpsWorkspace eps;  // workspace of the epsilon solve
  std::vector<TuneEntry> tuned;  // tile configurations that override the size rule
  unsigned* fs_words = nullptr;  // counters of the one-launch plain fixpoint (zero between launches)
  bool fs_dirty = false;         // a launch ended abnormally: clear them before the next
};

namespace dl {
void set_last_error(const std::string& m);
// Tile configuration of the product kernels for (prec, Np): the tuned entry
// if there is one, else the size rule of choose_nt_config.
int pick_config(const dl_ctx* c, int prec, int64_t np);
// The tuned or set entry for (prec, Np), -1 if there is none.
int tuned_config(const dl_ctx* c, int prec, int64_t np);
}  // namespace dl
