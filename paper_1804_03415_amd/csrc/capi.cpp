// C-ABI entry points (declared in include/mmdeig.h).  Each call converts
// exceptions into a status code and a thread-local message.
#include <algorithm>
#include <cstring>
#include <string>

#include "batch.h"
#include "handle.h"
#include "noalloc.h"
#include "solver.h"

namespace mmd {
namespace {
thread_local std::string g_last_error;
}
void set_last_error(const std::string& msg) { g_last_error = msg; }
const char* g_last_error_cstr() { return g_last_error.c_str(); }
}  // namespace mmd

namespace {

template <typename F>
int guarded(F&& f) {
  try {
    f();
    return MMD_OK;
  } catch (const mmd::Error& e) {
    mmd::set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    mmd::set_last_error("host allocation failed");
    return MMD_ENOMEM;
  } catch (const std::exception& e) {
    mmd::set_last_error(e.what());
    return MMD_EINVAL;
  }
}

eig_opts default_opts(const eig_opts* o) {
  eig_opts d;
  std::memset(&d, 0, sizeof(d));
  if (o) d = *o;
  return d;
}

}  // namespace

extern "C" {

int mmd_build(const mmd_csr* A, const mmd_build_opts* opts, void* hip_stream, mmd_handle** out) {
  return guarded([&] {
    MMD_REQUIRE(A && out, MMD_EINVAL, "null argument");
    MMD_REQUIRE(A->rowptr && A->colind && A->val, MMD_EINVAL, "null CSR array");
    mmd_build_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    auto* h = new mmd_handle();
    try {
      mmd::build_hierarchy(*h, *A, o);
      mmd::upload_hierarchy(*h, static_cast<hipStream_t>(hip_stream));
    } catch (...) {
      delete h;
      throw;
    }
    *out = h;
  });
}

int mmd_info(const mmd_handle* h, int32_t* K, int64_t* sizes, int64_t* nnzA, int64_t* nnzM,
             double* eps) {
  return guarded([&] {
    MMD_REQUIRE(h, MMD_EINVAL, "null handle");
    if (K) *K = h->K;
    for (int k = 0; k <= h->K; ++k) {
      if (sizes) sizes[k] = h->host[k].n;
      if (nnzA) nnzA[k] = h->host[k].A.nnz();
      if (nnzM) nnzM[k] = k == 0 ? 0 : h->host[k].M.nnz();
      if (eps) eps[k] = h->eps[k];
    }
  });
}

int mmd_export(const mmd_handle* h, int32_t level, int32_t which, int64_t* n_rows,
               int64_t* n_cols, int64_t* nnz, int64_t* rowptr, int32_t* colind, double* val) {
  return guarded([&] {
    MMD_REQUIRE(h, MMD_EINVAL, "null handle");
    MMD_REQUIRE(level >= 0 && level <= h->K, MMD_EINVAL, "level out of range");
    MMD_REQUIRE(which >= 0 && which <= 2, MMD_EINVAL, "which must be 0, 1 or 2");
    MMD_REQUIRE(which == 0 || level >= 1, MMD_EINVAL, "M and Psi exist for levels >= 1");
    const mmd::LevelHost& L = h->host[level];
    const mmd::HostCSR* src = which == 0 ? &L.A : (which == 1 ? &L.M : &L.Psi);
    mmd::HostCSR tmp;
    if (!h->perm.empty() && level == 0 && which == 0) src = &h->A_user;
    if (!h->perm.empty() && level == 1 && which == 2) {
      // rows of Psi^(1) are level-0 dofs: return them in the caller's numbering
      const mmd::HostCSR& P = L.Psi;
      const int n = P.n_rows;
      std::vector<int> iperm(n);
      for (int i = 0; i < n; ++i) iperm[h->perm[i]] = i;
      tmp.n_rows = P.n_rows;
      tmp.n_cols = P.n_cols;
      tmp.ptr.assign(n + 1, 0);
      for (int u = 0; u < n; ++u) tmp.ptr[u + 1] = tmp.ptr[u] + (P.ptr[iperm[u] + 1] - P.ptr[iperm[u]]);
      tmp.col.reserve(P.nnz());
      tmp.val.reserve(P.nnz());
      for (int u = 0; u < n; ++u)
        for (int64_t q = P.ptr[iperm[u]]; q < P.ptr[iperm[u] + 1]; ++q) {
          tmp.col.push_back(P.col[q]);
          tmp.val.push_back(P.val[q]);
        }
      src = &tmp;
    }
    const mmd::HostCSR& X = *src;
    if (n_rows) *n_rows = X.n_rows;
    if (n_cols) *n_cols = X.n_cols;
    if (nnz) *nnz = X.nnz();
    if (rowptr) {
      MMD_REQUIRE(colind && val, MMD_EINVAL, "null output array");
      std::copy(X.ptr.begin(), X.ptr.end(), rowptr);
      std::copy(X.col.begin(), X.col.end(), colind);
      std::copy(X.val.begin(), X.val.end(), val);
    }
  });
}

int eig_leftmost(mmd_handle* h, int32_t nev, double tol, const eig_opts* opts, double* evals,
                 double* evecs, eig_stats* st, void* hip_stream) {
  return guarded([&] {
    MMD_REQUIRE(h && evals && evecs, MMD_EINVAL, "null argument");
    mmd::Solver sv(*h, static_cast<hipStream_t>(hip_stream), default_opts(opts), st);
    sv.leftmost(nev, tol, evals, evecs);
  });
}

int eig_leftmost_batched(int32_t B, mmd_handle* const* hs, const int32_t* nev, double tol,
                         const eig_opts* opts, double* const* evals, double* const* evecs,
                         eig_stats* st, void* hip_stream) {
  return guarded([&] {
    mmd::leftmost_batched(B, hs, nev, tol, default_opts(opts), evals, evecs, st,
                          static_cast<hipStream_t>(hip_stream));
  });
}

int eig_backward(mmd_handle* h, int32_t nev, const double* evals, const double* evecs,
                 const double* g_evals, const double* g_evecs, double tol, double* g_vals,
                 void* hip_stream) {
  return guarded([&] {
    MMD_REQUIRE(h && evals && evecs && g_vals, MMD_EINVAL, "null argument");
    mmd::Solver sv(*h, static_cast<hipStream_t>(hip_stream), default_opts(nullptr), nullptr);
    sv.backward(nev, evals, evecs, g_evals, g_evecs, tol, g_vals);
  });
}

int mmd_apply(mmd_handle* h, int32_t level, int32_t op, const double* X, double* Y, int32_t b,
              void* hip_stream) {
  return guarded([&] {
    MMD_REQUIRE(h && X && Y, MMD_EINVAL, "null argument");
    mmd::Solver sv(*h, static_cast<hipStream_t>(hip_stream), default_opts(nullptr), nullptr);
    sv.apply_op(level, op, X, Y, b);
    MMD_HIP(hipStreamSynchronize(static_cast<hipStream_t>(hip_stream)));
  });
}

int mmd_solve(mmd_handle* h, int32_t level, int32_t kind, const double* rhs, double* X,
              int32_t b, int32_t use_x0, double tol, int32_t* iters, void* hip_stream) {
  return guarded([&] {
    MMD_REQUIRE(h && rhs && X, MMD_EINVAL, "null argument");
    mmd::Solver sv(*h, static_cast<hipStream_t>(hip_stream), default_opts(nullptr), nullptr);
    sv.solve(level, kind, rhs, X, b, use_x0 != 0, tol, iters);
  });
}

namespace {
// Shared body of mmdk_spmm and mmdk_spmm_noalloc: ptr32 receives the int32
// copy of the caller's row pointers (n_rows + 1 entries).
void spmm_caller_csr(int64_t n_rows, int64_t n_cols, const int64_t* rowptr, const int32_t* colind,
                     const double* val, const double* X, double* Y, int32_t b, hipStream_t s,
                     int* ptr32) {
  int64_t nnz = 0;
  MMD_HIP(hipMemcpyAsync(&nnz, rowptr + n_rows, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MMD_HIP(hipStreamSynchronize(s));
  MMD_REQUIRE(nnz >= 0 && nnz < (int64_t(1) << 31), MMD_EINVAL, "nnz out of range");
  mmd::i64_to_i32(rowptr, ptr32, n_rows + 1, s);
  mmd::CsrView A;
  A.n_rows = static_cast<int>(n_rows);
  A.n_cols = static_cast<int>(n_cols);
  A.nnz = nnz;
  A.rowptr = ptr32;
  A.col = colind;
  A.val = val;
  A.avg_row = n_rows ? static_cast<double>(nnz) / n_rows : 1.0;
  mmd::spmm(A, X, b, Y, b, b, s);
  MMD_HIP(hipStreamSynchronize(s));
}

void check_spmm_args(int64_t n_rows, int64_t n_cols, int32_t b) {
  MMD_REQUIRE(n_rows >= 0 && n_rows < (int64_t(1) << 31) && n_cols >= 0 &&
                  n_cols < (int64_t(1) << 31),
              MMD_EINVAL, "dimension out of range");
  MMD_REQUIRE(b > 0, MMD_EINVAL, "b must be positive");
}
}  // namespace

int mmdk_spmm(int64_t n_rows, int64_t n_cols, const int64_t* rowptr, const int32_t* colind,
              const double* val, const double* X, double* Y, int32_t b, void* hip_stream) {
  return guarded([&] {
    check_spmm_args(n_rows, n_cols, b);
    if (n_rows == 0) return;
    MMD_REQUIRE(rowptr && X && Y, MMD_EINVAL, "null argument");
    mmd::DBuf<int> ptr32(n_rows + 1);
    spmm_caller_csr(n_rows, n_cols, rowptr, colind, val, X, Y, b,
                    static_cast<hipStream_t>(hip_stream), ptr32.p);
  });
}

int mmdk_spmm_noalloc(int64_t n_rows, int64_t n_cols, const int64_t* rowptr,
                      const int32_t* colind, const double* val, const double* X, double* Y,
                      int32_t b, void* hip_stream) {
  return guarded([&] {
    check_spmm_args(n_rows, n_cols, b);
    MMD_REQUIRE(n_rows <= mmd::kNoAllocMaxRows, MMD_EINVAL,
                "mmdk_spmm_noalloc: n_rows exceeds the scratch capacity of 4194304 rows");
    if (n_rows == 0) return;
    MMD_REQUIRE(rowptr && X && Y, MMD_EINVAL, "null argument");
    spmm_caller_csr(n_rows, n_cols, rowptr, colind, val, X, Y, b,
                    static_cast<hipStream_t>(hip_stream), mmd::noalloc_scratch_rowptr32());
  });
}

int mmdk_gram(int64_t n, int32_t m, int32_t p, const double* X, int32_t ldx, const double* Y,
              int32_t ldy, double* C, int32_t ldc, void* hip_stream) {
  return guarded([&] {
    MMD_REQUIRE(n >= 0 && n < (int64_t(1) << 31) && m >= 0 && p >= 0, MMD_EINVAL,
                "dimension out of range");
    MMD_REQUIRE(ldx >= m && ldy >= p && ldc >= p, MMD_EINVAL, "leading dimension too small");
    if (m == 0 || p == 0) return;
    MMD_REQUIRE(C && (n == 0 || (X && Y)), MMD_EINVAL, "null argument");
    const auto s = static_cast<hipStream_t>(hip_stream);
    mmd::DBuf<double> work(std::max<size_t>(1, mmd::gram_work_size(static_cast<int>(n), m, p)));
    mmd::gram(X, ldx, Y, ldy, static_cast<int>(n), m, p, C, ldc, work.p, s);
    MMD_HIP(hipStreamSynchronize(s));
  });
}

int mmdk_gemm(int64_t n, int32_t m, int32_t p, double alpha, const double* X, int32_t ldx,
              const double* Cm, int32_t ldc, double beta, double* Z, int32_t ldz,
              void* hip_stream) {
  return guarded([&] {
    MMD_REQUIRE(n >= 0 && n < (int64_t(1) << 31) && m >= 0 && p >= 0, MMD_EINVAL,
                "dimension out of range");
    MMD_REQUIRE(ldx >= m && ldc >= p && ldz >= p, MMD_EINVAL, "leading dimension too small");
    if (n == 0 || p == 0) return;
    MMD_REQUIRE(Z && (m == 0 || (X && Cm)), MMD_EINVAL, "null argument");
    const auto s = static_cast<hipStream_t>(hip_stream);
    mmd::gemm_nn(X, ldx, Cm, ldc, Z, ldz, static_cast<int>(n), m, p, alpha, beta, s);
    MMD_HIP(hipStreamSynchronize(s));
  });
}

void mmd_free(mmd_handle* h) { delete h; }

const char* mmd_last_error(void) { return mmd::g_last_error_cstr(); }

}  // extern "C"
