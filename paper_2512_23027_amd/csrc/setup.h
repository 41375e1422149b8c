// Host-side problem setup for the SG wave solver: Hermite-chaos Galerkin
// tensor, KLE and log-normal PCE of the squared wave speed, structured P1
// mesh, rectilinear domain decomposition, SG matrix assembly in sliced-ELL
// form and the nested-dissection Cholesky factors of the mean subdomain
// matrices.  Pure C++ (no HIP); sgw.cpp uploads the result.
#pragma once
#include <string>
#include <vector>

#include "sgw.h"

namespace sgw {

// Galerkin tensor c_kij = <psi_k psi_i psi_j> of the normalised Hermite chaos
// (Eq. galerproject_chap2), k over the input basis (|a| <= p_in), i, j over
// the output basis (|a| <= p_out).  Stored as a list of nonzeros.
struct Galerkin {
  int L = 0, p_in = 0, p_out = 0, nk = 0, P = 0;
  std::vector<std::vector<int>> in_idx, out_idx;  // multi-indices
  std::vector<int> k, i, j;                       // nonzero entries
  std::vector<double> v;
};
Galerkin build_galerkin(int L, int p_in, int p_out);

// Sliced-ELL sparse matrix: W slots per row, column-major over rows so that
// consecutive rows of one slot are contiguous.  col[s * nrows + r];
// val[(k * W + s) * nrows + r] for the nk PCE coefficient matrices;
// mval[s * nrows + r] for the (deterministic) mass matrix.  Unused slots have
// col = r and value 0.
struct Ell {
  int nrows = 0, W = 0, nk = 0;
  std::vector<int> col;
  std::vector<double> val;
  std::vector<double> mval;
};

// Batched mean-matrix Cholesky factors, one block per subdomain, in the
// supernodal pull form used by the triangular-solve kernel.  Rows of block b
// are [row_off[b], row_off[b+1]) of the system; inside a block they are in
// nested-dissection order, every supernode is one nested-dissection set
// (leaf box or separator) and its diagonal block is stored as the dense
// inverse of the Cholesky diagonal block.
struct Factor {
  int nb = 0;
  std::vector<int> row_off;            // nb + 1
  std::vector<int> lvl_off;            // nb + 1, into lvl_ptr (nlev+1 each)
  std::vector<int> lvl_ptr;            // supernode ranges per level
  std::vector<int> lrow_ptr;           // row ranges per level (same indexing)
  std::vector<int> lrow_list, lrow_sn; // local rows of each level, their supernode
  std::vector<int> lvl_gf, lvl_gb;     // lanes per row of the forward/backward pulls
  std::vector<int> sn_beg, sn_w, sn_dinv;  // local first row, width, dinv offset
  // off-diagonal L by level-list position (global positions, one pointer
  // array over all blocks): row entries (local columns) and column entries
  // (local rows)
  std::vector<int> lr_ptr, lr_col;
  std::vector<double> lr_val;
  std::vector<int> lc_ptr, lc_row;
  std::vector<double> lc_val;
  std::vector<double> dinv;            // dense w x w inverse blocks, row-major
  std::vector<double> dinvT;           // the same blocks column-major
  int max_rows = 0, max_level_rows = 0, max_w = 0, max_levels = 0, max_sn = 0;
  int max_lvl_d = 0;                   // largest sum of w^2 over one level
  long long nnz_l = 0;
};

struct Host {
  sgw_problem_desc d{};
  std::vector<int> xs, ys;
  int n = 0, nn = 0, nsub = 0;
  Galerkin g;
  double a_m = 0, s_k = 0;     // K~_0 = a_m M + s_k K_0, K~_k = s_k K_k
  // DD numbering of the free nodes: interior blocks of the subdomains, then
  // the interface nodes (sorted by mesh index).
  int NF = 0, nI = 0, nG = 0, nC = 0, NT = 0;
  std::vector<int> dd2mesh, mesh2dd;   // mesh2dd = -1 on the boundary
  std::vector<int> Ioff, Toff;         // nsub + 1
  std::vector<int> torn2dd;            // torn (Neumann) row -> dd index
  Ell glob, dir, neu;
  Factor fD, fN;
  // Chebyshev interval (lo, hi) of the Jacobi-scaled mean matrix per block
  std::vector<double> chebD, chebN;
  // D_s R_s: for every torn row, interface index (or -1) and weight 1/mult
  std::vector<int> torn_gidx;
  std::vector<double> torn_w;
  // sum_s R_s^T D_s: for every interface node, the torn copies and weights
  std::vector<int> gam_ptr, gam_torn;
  std::vector<double> gam_w;
  std::vector<int> g2c;                // interface index -> coarse index / -1
  std::vector<int> c2g;                // coarse index -> interface index
  // corners of each subdomain
  std::vector<int> sc_ptr, sc_coarse, sc_gidx;
  std::vector<double> sc_w;
  // local Neumann matrix rows of every subdomain corner: couplings to the
  // subdomain's torn rows (K~^s_k[c, t], nk values per entry) and self terms
  std::vector<int> cc_ptr, cc_torn;
  std::vector<double> cc_val, cself;
  // KLE / PCE diagnostics
  std::vector<double> kle_lambda;
  std::vector<double> kappa;           // [nk][ne]
};

// Returns 0 or a negative SGW_* code with a message in err.
int build_host(const sgw_problem_desc& d, Host& h, std::string& err);

}  // namespace sgw
