// Context of the C ABI (shared by borth.cpp and batch.cpp; host only).
#pragma once
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/borth.h"
#include "internal.hpp"
#include "noalloc.hpp"

struct GraphKey {
  std::vector<int64_t> v;
  bool operator<(const GraphKey& o) const { return v < o.v; }
};

// A double as a cache-key entry: its bit pattern (defined for every value,
// unlike a scaled integer conversion).
inline int64_t key_bits(double x) {
  int64_t b;
  std::memcpy(&b, &x, sizeof b);
  return b;
}

struct TimedPair {
  hipEvent_t a, b;
};

struct borth_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  double* part = nullptr;
  int64_t part_cap = 0;  // doubles
  double* ws = nullptr;
  int64_t ws_cap = 0;
  int* status = nullptr;   // device, 4 ints (+ batch statuses)
  int status_cap = 0;
  int* h_status = nullptr;  // pinned host copy
  int h_status_cap = 0;
  std::map<GraphKey, hipGraphExec_t> graphs;
  uint64_t ws_generation = 0;
  // profiling
  int prof = 0;  // mask of timed kinds: 1 Gram sweeps, 2 update sweeps
  std::vector<TimedPair> ev_free;
  std::vector<TimedPair> ev_used[2];
  // autotune table: key (mode, kp, ky>0) -> tune
  std::map<std::tuple<int, int, int>, borth::TuneGram> tune_gram;
  std::map<std::tuple<int, int, int>, borth::TuneGram> tune_upd;
  // batched calls: plans (descriptor tables, workspace, captured graph)
  std::map<GraphKey, struct BatchPlan*> plans;
  uint64_t tune_generation = 0;
  hipStream_t cap_stream = nullptr;  // private stream for graph capture
  bool capturing = false;
  bool last_est = false;             // the last call left estimates in the workspace
  hipStream_t cur = nullptr;         // stream the current enqueue targets
  std::string noalloc_err;           // set if the scratch address could not be taken
};

inline borth_status fail_hip(borth_ctx c, hipError_t e, const char* where) {
  if (c) {
    c->err = std::string(where) + ": " + hipGetErrorString(e);
  }
  return BORTH_ERR_HIP;
}

inline borth_status fail_arg(borth_ctx c, const char* what) {
  if (c) c->err = std::string("invalid argument: ") + what;
  return BORTH_ERR_ARG;
}

#define HIPCHK(c, expr, where)                 \
  do {                                         \
    hipError_t _e = (expr);                    \
    if (_e != hipSuccess) return fail_hip(c, _e, where); \
  } while (0)

// Largest workgroup count of a single-block sweep (default 1024; the
// autotuner may pick up to this many); partial buffers are sized for it.
constexpr int64_t kMaxSweepWG = 4096;

inline int pow2pad(int k) {
  int p = 4;
  while (p < k) p <<= 1;
  return p;
}

inline borth::TuneGram lookup(const std::map<std::tuple<int, int, int>, borth::TuneGram>& t, int mode, int kp,
                       int hasy) {
  auto it = t.find(std::make_tuple(mode, kp, hasy));
  if (it != t.end()) return it->second;
  return borth::TuneGram{0, 0};
}

// Profiling: HIP events around the dominant launches (kind 0 Gram sweeps,
// kind 1 update sweeps) on the stream they run on; skipped under capture.
inline void prof_begin(borth_ctx c, int kind) {
  if (!(c->prof & (1 << kind)) || c->capturing) return;
  TimedPair p;
  if (!c->ev_free.empty()) {
    p = c->ev_free.back();
    c->ev_free.pop_back();
  } else {
    hipEventCreate(&p.a);
    hipEventCreate(&p.b);
  }
  hipEventRecord(p.a, c->cur);
  c->ev_used[kind].push_back(p);
}
inline void prof_end(borth_ctx c, int kind) {
  if (!(c->prof & (1 << kind)) || c->capturing) return;
  hipEventRecord(c->ev_used[kind].back().b, c->cur);
}

// Batched path (batch.cpp): releases every cached plan.
void batch_free_all(borth_ctx c);
