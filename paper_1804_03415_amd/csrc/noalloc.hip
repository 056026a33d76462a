// Library-owned device scratch for the entry points that must not allocate
// (callers under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).  The buffer is a file-scope device array: every GPU the
// library runs on holds one copy from module load until the process ends.
//
// In host code the array's name is only a stand-in for the device symbol;
// its device address is looked up once per device with hipGetSymbolAddress
// (with that device current) and only that address is ever handed to
// kernels or copies.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "common.h"
#include "noalloc.h"

namespace mmd {

namespace {

// int32 row pointers of a caller CSR with at most kNoAllocMaxRows rows (16 MiB)
__device__ __align__(256) int scratch[kNoAllocMaxRows + 1];

std::mutex g_mu;
std::map<int, int*> g_addr;  // device ordinal -> address of scratch on it

}  // namespace

int* noalloc_scratch_rowptr32() {
  int dev = 0;
  MMD_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(g_mu);
  auto it = g_addr.find(dev);
  if (it != g_addr.end()) return it->second;
  void* p = nullptr;
  MMD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  MMD_REQUIRE(p != nullptr, MMD_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
  int* ip = static_cast<int*>(p);
  g_addr.emplace(dev, ip);
  return ip;
}

}  // namespace mmd
