// The decomposition handle: host copies of every level (used by the host
// builder, the coarsest-level dense solve and mmd_export) and the device
// operators the solver runs on.
#pragma once

#include <cstdint>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "mixed.h"

namespace mmd {

struct HostCSR {
  int n_rows = 0, n_cols = 0;
  std::vector<int64_t> ptr;
  std::vector<int> col;
  std::vector<double> val;
  int64_t nnz() const { return ptr.empty() ? 0 : ptr.back(); }
};

struct LevelHost {
  int n = 0;
  HostCSR A;        // A^(k) (level 0: the input matrix)
  HostCSR M;        // M^(k), k >= 1 (level 0: identity, left empty)
  HostCSR Psi;      // Psi^(k): N^(k-1) x N^(k), k >= 1
  // transfer k-1 -> k: patches of level-(k-1) dofs and their reflectors
  std::vector<int> patch_ptr, members;
  std::vector<double> hh_u, hh_scale, phi;
  std::vector<double> eps_patch;
  double eps_level = 0.0;   // eps(P^(k))
  double lam_max_M = 1.0;   // Gershgorin bound of lambda_max(M^(k))
  std::vector<double> coords;
  int cdim = 0;
  std::vector<int> grid;    // coarse grid shape (empty: not a grid)
  // level 0 only: edge form
  std::vector<double> s;    // self-loop weights
};

struct LevelDev {
  DBuf<int> a_ptr, a_col, m_ptr, m_col, p_ptr, p_col, h_ptr, h_mem;
  DBuf<double> a_val, a_diag, m_val, p_val, h_u, h_scale;
  DBuf<int> t_row, t_uptr, t_urow;  // level-0 row-block tiling (kernels.h)
  DBuf<unsigned short> t_lcol;
  CsrView A, M, Psi;
  HouseView H;  // transfer (k-1 -> k): U^(k)
  // FP32 copy of A (level 0, mixed precision), made on first use
  DBuf<float> a_val32, a_diag32;
  CsrView32 A32;
  bool has32 = false;
};

}  // namespace mmd

struct mmd_handle {
  int64_t n = 0;
  int K = 0;
  // Level 0 is stored renumbered patch by patch (Morton order of the patches):
  // internal index i holds caller index perm[i].  Empty: identity.
  std::vector<int> perm;
  mmd::DBuf<int> d_perm;
  mmd::HostCSR A_user;  // the caller's matrix in its own numbering (export)
  // the caller's CSR pattern on the device (eigen-backward output order), made
  // on first use
  mmd::DBuf<int> u_ptr, u_col;
  bool has_upat = false;
  std::vector<mmd::LevelHost> host;
  std::vector<mmd::LevelDev> dev;
  std::vector<double> eps;  // cumulative eps_k, eps[0] = 0
};

namespace mmd {
// host builder (mmd_build.cpp)
void build_hierarchy(mmd_handle& h, const mmd_csr& A, const mmd_build_opts& o);
void upload_hierarchy(mmd_handle& h, hipStream_t s);
}  // namespace mmd
