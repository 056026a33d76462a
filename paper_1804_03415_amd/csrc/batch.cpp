// Batched eigensolves: many independent problems, each a full Alg. 6 run
// (host-driven control flow, many small kernels and host round trips), are
// overlapped by running several of them at once on separate HIP streams, one
// host thread per stream.  Problems are handed out largest first (nnz x nev),
// so the long ones start early and the short ones fill the tail.  The
// persistent single-vector solvers run one at a time across the batch (a
// process-wide lock around each launch), everything else overlaps freely.
#include <algorithm>
#include <atomic>
#include <mutex>
#include <numeric>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "batch.h"
#include "solver.h"

namespace mmd {

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
          sv.set_serialize_persistent(true);
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
    if (s) (void)hipStreamDestroy(s);
  };
  std::vector<std::thread> pool;
  pool.reserve(T);
  for (int t = 0; t < T; ++t) pool.emplace_back(worker);
  for (auto& th : pool) th.join();
  (void)hipEventDestroy(start);
  if (err_code != MMD_OK) throw Error(err_code, err_msg);
}

}  // namespace mmd
