// Batched eig_leftmost over independent decompositions (see batch.cpp).
#pragma once

#include <hip/hip_runtime_api.h>

#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <string>

#include "handle.h"
#include "mmdeig.h"
#include "pcg_persistent.h"

namespace mmd {

void leftmost_batched(int B, mmd_handle* const* hs, const int* nev, double tol,
                      const eig_opts& o, double* const* evals, double* const* evecs,
                      eig_stats* st, hipStream_t caller);

// Merges the single-vector operator solves (Section 4, OP) that the problems
// of a batch request concurrently into cooperative launches of the batched
// persistent kernel: each launch runs every pending request on its own block
// range.  The calling worker threads take turns as the leader that collects
// requests (until every active worker has one pending, or a short window has
// passed), launches them on the batcher's stream and waits; the others sleep
// until their request is solved.
class OpBatcher {
 public:
  explicit OpBatcher(int workers);
  ~OpBatcher();
  OpBatcher(const OpBatcher&) = delete;
  OpBatcher& operator=(const OpBatcher&) = delete;
  // Solve r (its right-hand side must already be complete on the device);
  // returns when the batch holding r has finished.
  void solve(const Pcg1Req& r);
  // The calling worker has no further problems.
  void leave();
  int64_t launches() const { return launches_; }
  int64_t requests() const { return requests_; }

 private:
  struct Slot {
    const Pcg1Req* req;
    bool done = false;
    int err = 0;
    std::string msg;
  };
  void lead(std::unique_lock<std::mutex>& lk);
  int capacity(size_t lds);
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<Slot*> pending_;
  int active_;
  bool leading_ = false;
  hipStream_t s_ = nullptr;
  DBuf<Pcg1Req> d_;
  HBuf<Pcg1Req> h_;
  std::map<size_t, int> cap_;
  int64_t launches_ = 0, requests_ = 0;
};

}  // namespace mmd
