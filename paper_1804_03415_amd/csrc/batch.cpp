// Batched eigensolves: many independent problems, each a full Alg. 6 run
// (host-driven control flow, many small kernels and host round trips), are
// overlapped by running several of them at once on separate HIP streams, one
// host thread per stream.  Problems are handed out largest first (nnz x nev),
// so the long ones start early and the short ones fill the tail.  The
// single-vector operator solves of all problems go through one OpBatcher,
// which runs the ones pending at the same time in one cooperative launch of
// the batched persistent kernel (each on its own block range); everything else
// overlaps on the problems' streams.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <numeric>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "batch.h"
#include "solver.h"

namespace mmd {

OpBatcher::OpBatcher(int workers) : active_(workers) {
  MMD_HIP(hipStreamCreateWithFlags(&s_, hipStreamNonBlocking));
}

OpBatcher::~OpBatcher() {
  if (s_) (void)hipStreamDestroy(s_);
}

int OpBatcher::capacity(size_t lds) {
  auto it = cap_.find(lds);
  if (it == cap_.end()) it = cap_.emplace(lds, pcg1_multi_capacity(lds)).first;
  return it->second;
}

void OpBatcher::leave() {
  std::lock_guard<std::mutex> g(mu_);
  --active_;
  cv_.notify_all();
}

void OpBatcher::solve(const Pcg1Req& r) {
  Slot me{&r};
  std::unique_lock<std::mutex> lk(mu_);
  pending_.push_back(&me);
  cv_.notify_all();  // a waiting leader may now hold a full batch
  while (!me.done) {
    if (!leading_) {
      leading_ = true;
      lead(lk);
      leading_ = false;
      cv_.notify_all();
    } else {
      cv_.wait(lk);
    }
  }
  if (me.err) throw Error(me.err, me.msg);
}

void OpBatcher::lead(std::unique_lock<std::mutex>& lk) {
  // collect: until every active worker has a request pending, or the window
  // (short against one solve, ~1 ms and more) has passed
  const auto t0 = std::chrono::steady_clock::now();
  const auto window = std::chrono::microseconds(150);
  while (static_cast<int>(pending_.size()) < active_) {
    const auto left = window - (std::chrono::steady_clock::now() - t0);
    if (left <= std::chrono::steady_clock::duration::zero()) break;
    cv_.wait_for(lk, left);
  }
  std::vector<Slot*> batch;
  std::vector<Pcg1Req> reqs;
  int blocks = 0;
  size_t lds = 0;
  while (!pending_.empty()) {
    Slot* sl = pending_.front();
    const int nb = (sl->req->nblk + 7) / 8 * 8;
    const size_t l = std::max(lds, sl->req->lds);
    lk.unlock();
    int cap = 0;
    try {
      cap = capacity(l);
    } catch (...) {
      cap = 0;
    }
    lk.lock();
    // the first request always goes: its own plan was checked for co-residency
    if (!batch.empty() && blocks + nb > cap) break;
    pending_.pop_front();
    batch.push_back(sl);
    reqs.push_back(*sl->req);
    blocks += nb;
    lds = l;
  }
  if (batch.empty()) return;
  lk.unlock();
  int err = 0;
  std::string msg;
  try {
    h_.ensure(reqs.size());
    d_.ensure(reqs.size());
    pcg1_multi(reqs, h_.p, d_.p, s_);
    MMD_HIP(hipStreamSynchronize(s_));
  } catch (const Error& e) {
    err = e.code;
    msg = e.what();
  } catch (const std::exception& e) {
    err = MMD_EHIP;
    msg = e.what();
  }
  lk.lock();
  ++launches_;
  requests_ += static_cast<int64_t>(batch.size());
  for (Slot* sl : batch) {
    sl->done = true;
    sl->err = err;
    sl->msg = msg;
  }
  cv_.notify_all();
}

void leftmost_batched(int B, mmd_handle* const* hs, const int* nev, double tol,
                      const eig_opts& o, double* const* evals, double* const* evecs,
                      eig_stats* st, hipStream_t caller) {
  MMD_REQUIRE(B >= 0, MMD_EINVAL, "negative batch size");
  if (B == 0) return;
  MMD_REQUIRE(hs && nev && evals && evecs, MMD_EINVAL, "null argument");
  {
    std::set<const mmd_handle*> seen;
    for (int b = 0; b < B; ++b) {
      const std::string who = "problem " + std::to_string(b) + ": ";
      MMD_REQUIRE(hs[b], MMD_EINVAL, who + "null handle");
      MMD_REQUIRE(nev[b] > 0 && nev[b] <= hs[b]->n, MMD_EINVAL, who + "nev out of range");
      MMD_REQUIRE(evals[b] && evecs[b], MMD_EINVAL, who + "null output buffer");
      MMD_REQUIRE(seen.insert(hs[b]).second, MMD_EINVAL, who + "handle appears twice in the batch");
    }
  }
  std::vector<int> order(B);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const double wa = static_cast<double>(hs[a]->host[0].A.nnz()) * nev[a];
    const double wb = static_cast<double>(hs[b]->host[0].A.nnz()) * nev[b];
    return wa > wb;
  });
  const int T = std::max(1, std::min(B, o.streams > 0 ? o.streams : 8));
  // the batch starts after the caller's earlier work
  hipEvent_t start;
  MMD_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
  MMD_HIP(hipEventRecord(start, caller));
  int dev = 0;
  MMD_HIP(hipGetDevice(&dev));
  std::atomic<int> next{0};
  std::mutex mu;
  int err_code = MMD_OK;
  std::string err_msg;
  auto fail = [&](int code, const std::string& msg) {
    std::lock_guard<std::mutex> g(mu);
    if (err_code == MMD_OK) {
      err_code = code;
      err_msg = msg;
    }
  };
  OpBatcher batcher(T);
  auto worker = [&]() {
    hipStream_t s = nullptr;
    try {
      MMD_HIP(hipSetDevice(dev));
      MMD_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      MMD_HIP(hipStreamWaitEvent(s, start, 0));
      for (int i = next++; i < B; i = next++) {
        const int b = order[i];
        try {
          Solver sv(*hs[b], s, o, st ? &st[b] : nullptr);
          sv.set_batcher(&batcher);
          sv.leftmost(nev[b], tol, evals[b], evecs[b]);
        } catch (const Error& e) {
          fail(e.code, "problem " + std::to_string(b) + ": " + e.what());
        } catch (const std::bad_alloc&) {
          fail(MMD_ENOMEM, "problem " + std::to_string(b) + ": host allocation failed");
        } catch (const std::exception& e) {
          fail(MMD_EINVAL, "problem " + std::to_string(b) + ": " + e.what());
        }
      }
      MMD_HIP(hipStreamSynchronize(s));
    } catch (const Error& e) {
      fail(e.code, e.what());
    }
    batcher.leave();
    if (s) (void)hipStreamDestroy(s);
  };
  std::vector<std::thread> pool;
  pool.reserve(T);
  for (int t = 0; t < T; ++t) pool.emplace_back(worker);
  for (auto& th : pool) th.join();
  (void)hipEventDestroy(start);
  if (const char* e = std::getenv("MMDEIG_LOG"))
    if (e[0] && e[0] != '0')
      std::fprintf(stderr, "[mmdeig] batch: %lld operator solves in %lld batched launches\n",
                   (long long)batcher.requests(), (long long)batcher.launches());
  if (err_code != MMD_OK) throw Error(err_code, err_msg);
}

}  // namespace mmd
