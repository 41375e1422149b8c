// Launchers of the HIP kernels of the SG wave solver (gfx950).
// Vectors are mode-major: element (mode j, row r) of a vector with leading
// dimension ld sits at v[j * ld + r].
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace sgw {
namespace k {

// Galerkin contraction table of the SG operator apply, for one (nk, P,
// chunk KC, output group GS) choice.  For output group g, k-chunk ch and
// input mode j: mask bit kk says that coefficient matrix ch*KC+kk meets mode
// j with some output i of group g; for every set bit, in order, pair_cnt
// gives the number of (i, c) entries, stored consecutively in ent_i / ent_c.
struct GTab {
  int nk = 0, P = 0, KC = 0, GS = 0, ng = 0, nch = 0;
  int L = -1, p_in = -1, p_out = -1;  // basis, for the specialised kernels
  bool use_spec = true;              // false: always the table-driven kernel
  const uint32_t* mask = nullptr;    // [ng][nch][P]
  const int* pair_beg = nullptr;     // [ng][nch][P]
  const int* ent_beg = nullptr;      // [ng][nch][P]
  const int* pair_cnt = nullptr;
  const int* ent_i = nullptr;        // output mode within the group
  const double* ent_c = nullptr;
  const float* ent_cf = nullptr;
};

// Sliced-ELL matrix on the device (see setup.h): col[s*nrows + r],
// val[(k*W + s)*nrows + r], mval[s*nrows + r].
template <typename T>
struct DEll {
  int nrows = 0, W = 0, nk = 0;
  const int* col = nullptr;
  const T* val = nullptr;
  const T* mval = nullptr;
};

// Column halo of the row groups (at most 64 rows each) of a sliced-ELL
// matrix, for rows [r0, r0 + nr): group g covers rows [grow[g], grow[g+1])
// and its distinct columns are idx[ptr[g] .. ptr[g+1]) (sorted);
// lcol[s*nr + r - r0] is the position of col[s][r] in its group's list;
// hmax = the longest list.  Either plain 64-row chunks (aligned64), or
// groups that never straddle the blocks of a block-diagonal system: then
// gblk[g] = block of group g and bgrp[b] = first group of block b.
struct DHalo {
  int r0 = 0, nr = 0, hmax = 0, ng = 0;
  bool aligned64 = true;
  const int* ptr = nullptr;
  const int* idx = nullptr;
  const unsigned short* lcol = nullptr;
  const int* grow = nullptr;
  const int* gblk = nullptr;
  const int* bgrp = nullptr;
};
// workgroups (row groups) covering rows [r0, r0 + nrows) of a halo starting at r0
inline int halo_groups(const DHalo& H, int r0, int nrows) {
  if (r0 != H.r0 || nrows > H.nr) return -1;
  if (nrows == H.nr) return H.ng;
  return H.aligned64 ? (nrows + 63) / 64 : -1;
}

// y[i][r] = alpha * sum_k sum_j c_kij sum_s K_k[r, s] x[j][col]  (+ beta*y)
// for rows r in [r0, r0 + nrows) of the matrix.  nbatch vectors with strides.
// With a halo H of the same r0 covering the rows (and a generated kernel
// for the basis) the kernel that stages x in LDS runs, else the
// table-driven one.
template <typename T>
void sg_apply(const DEll<T>& A, const GTab& g, const DHalo* H, int r0, int nrows,
              const T* x, int ldx, T* y, int ldy, T alpha, T beta,
              int nbatch, long long sx, long long sy, hipStream_t st);
// Once per process before the first sg_apply: LDS attribute of the
// generated kernels.  0 on success, -1 on a HIP error.
int sg_apply_prepare();
// number of generated (unrolled-tensor) kernels for the basis in a precision
// (wbytes = 4 or 8 bytes per value), one per group of output modes; 0 if
// none is generated
int sg_apply_generated(int L, int p_in, int p_out, int wbytes);
// whether the generated PCG variant of the basis exists for precision T and
// its LDS (staged tile of the halo, wave partials) fits the halo H
template <typename T>
bool sg_apply_pcg_fits(const GTab& g, const DHalo& H);
// The SG apply of one subdomain PCG iteration on a block-aligned halo (all
// nrows rows): p = z + beta_b pold (beta_b = new r'z of block b from rzpart
// over its old r'z in sc[b*8 + 1 - par], 0 if that is infinite; the new r'z
// goes to sc[b*8 + par]), pnew = p on every row, q = K~ p, and
// pqg[g*K + k] = p'q over the rows of group g and the output modes of
// generated kernel k (K = sg_apply_generated(...)).  With acct != null every
// active row group adds its rows times bpr (algorithmic bytes per row) to
// *acct.  Returns false (nothing launched) if
// no generated kernel fits.
template <typename T>
bool sg_apply_pcg(const DEll<T>& A, const GTab& g, const DHalo& H, int nrows, const T* pold,
                  const T* z, T* pnew, int ld, T* q, const double* rzpart, double* sc, int par,
                  double* pqg, unsigned long long* acct, unsigned bpr, hipStream_t st);

// y[j][r] = beta*y[j][r] + alpha * sum_s M[r, s] x[j][col]  for all P modes.
template <typename T>
void mass_apply(const DEll<T>& A, int r0, int nrows, int P, const T* x,
                int ldx, T* y, int ldy, T alpha, T beta, hipStream_t st);

// Batched supernodal triangular solves with the mean-matrix factor:
// out = (L L^T)^{-1} rhs for every block and P modes (nbatch vectors).
struct DFactor {
  int nb = 0, P = 0;
  const int *row_off, *lvl_off, *lvl_ptr, *lrow_ptr, *lrow_list, *lrow_sn;
  const int *sn_beg, *sn_w, *sn_dinv, *lr_ptr, *lr_col, *lc_ptr, *lc_row;
  const int *lvl_gf, *lvl_gb;  // lanes per row in the pull phases (0: no entries)
  const double *lr_val, *lc_val, *dinv, *dinvT;  // dinv row-major, dinvT column-major
  const float *lr_valf, *lc_valf, *dinvf, *dinvTf;
  int max_rows = 0, max_level_rows = 0, max_sn = 0, max_levels = 0, max_lvl_d = 0;
  const int* order = nullptr;  // launch order of the blocks (largest first), may be null
};
template <typename T>
size_t tri_lds_bytes(const DFactor& f, int Q);
template <typename T>
void tri_solve(const DFactor& f, int Q, const T* rhs, int ldr, T* out,
               int ldo, int nbatch, long long sr, long long so, hipStream_t st);

// Chebyshev polynomial preconditioner (degree deg, Q modes per workgroup,
// launch shape 0, 1, 2 = 1024, 512, 256 threads per workgroup with 1, 2 or 4
// rows per thread) on the blocks of the mean matrix; coef[b * 2 deg ...] =
// the iteration coefficients of block b (cheb_coefficients); order (may be
// null) = launch order of the blocks (largest first); crow[r0 + i] = system
// row at natural (lexicographic) position i of the block starting at r0;
// [8]-records by natural position r0 + i: cnb[8 (r0 + i) + s] = natural
// position of that row's slot-s neighbour within the block (slot 0: the row
// itself), cval[8 (r0 + i) + s] = its mean-matrix value (slots 7 and
// unused ones: value 0, position of the row itself).  Writes z and
// part[b*P + j] = r_j'z_j (part2 = r_j'r_j if not null).  With sc != null it
// first does the PCG stopping test of iteration par (r'r from rrpart, see
// pcg_test) and skips converged blocks.  With acct != null, every active workgroup adds its algorithmic
// bytes (right-hand sides in and out, the block's mean matrix once) to
// *acct.  With ev0 and ev1 the launch records them with the kernel's
// dispatch (hipExtLaunchKernelGGL).  Returns -1 (nothing
// launched) if Q, the shape, deg or the block
// size is out of range (max_rows <= 4 x the workgroup size, Q <= cheb_max_q,
// deg <= 64, cheb_lds_bytes <= 150 KiB).
template <typename T>
size_t cheb_lds_bytes(int max_rows, int Q, int shape);
// Coefficients of deg Chebyshev steps on the spectral interval [lo, hi] of
// one block (Saad, Alg. 12.1), in the layout cheb_apply reads: out[0] =
// 1/theta, out[1] = 0, out[2k] = rho_k rho_{k-1}, out[2k+1] = 2 rho_k / delta
// for k = 1..deg-1 (theta, delta: centre and half width of the interval,
// the half width at least 1e-3 theta; rho_0 = delta / theta,
// rho_k = 1 / (2 theta / delta - rho_{k-1})).  Computed in double.
void cheb_coefficients(double lo, double hi, int deg, double* out);
// largest mode tile cheb_apply accepts for blocks of up to max_rows rows
// with the given shape (0: the shape does not cover such blocks)
template <typename T>
int cheb_max_q(int max_rows, int shape);
// Once per process before the first cheb_apply: allows the kernels the full
// 160 KiB of LDS.  0 on success, -1 on a HIP error.
int cheb_prepare();
template <typename T>
int cheb_apply(const T* cval, const int* row_off, const int* order, const int* crow,
               const unsigned short* cnb, const T* coef, int nb, int P, int deg,
               int Q, int shape, int max_rows, const T* r, int ldr, T* z, int ldz,
               double* part, double* part2, double* sc, int par, double tol2,
               const double* rrpart, int* flags, unsigned long long* acct, hipStream_t st,
               hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// Segmented dot products: partial[b * P + j] = sum_{r in block b} a[j][r] b[j][r]
// (row_off relative to the vectors; a second vector pair is optional).
template <typename T>
void seg_dot(int nb, const int* row_off, int P, const T* a, int lda,
             const T* b, int ldb, double* partial, const T* c, int ldc,
             const T* d, int ldd, double* partial2, hipStream_t st);

// Batched block PCG bookkeeping (per-block scalars sc[b*8], parity slots
// by iteration index, see kernels.hip).
// start: r'z (part), r'r = b'b (part2), initial stopping test
void pcg_start(int nb, int P, const double* part, const double* part2, double* sc,
               double tol2, double negl, int* flags, hipStream_t st);
// x += alpha_b p ; r -= alpha_b q with alpha_b = r'z / p'q (p'q from part);
// part2[b*P + j] = ||r_bj||^2 on the active blocks; flags[3] = the largest
// number of iterations a block has taken (flags has 4 entries)
// (with bgrp: p'q summed from the partials part[g*pqn + k], k < pqn, of the
// block's groups g = bgrp[b] .. bgrp[b+1]-1)
template <typename T>
void pcg_xr(int nb, const int* row_off, int P, int par, double* sc, T* x, int ldx,
            const T* p, int ldp, T* r, int ldr, const T* q, int ldq, const double* part,
            double* part2, int* flags, hipStream_t st, const int* bgrp = nullptr,
            int pqn = 0);
// stopping test of iteration par from part2 (exact-preconditioner path)
void pcg_test(int nb, int P, int par, const double* part2, double* sc, double tol2,
              int* flags, hipStream_t st);
// p = z + beta_b p with beta_b = (r'z from part) / (previous r'z)
template <typename T>
void pcg_p(int nb, const int* row_off, int P, int par, double* sc, const double* part,
           const T* z, int ldz, T* p, int ldp, hipStream_t st);

// strided copies / fills over [P][n] (dst = a*src, optional type change)
template <typename TD, typename TS>
void copy2d(int P, int n, const TS* src, int lds, TD* dst, int ldd, double a,
            hipStream_t st);
template <typename T>
void fill2d(int P, int n, T* dst, int ldd, T v, hipStream_t st);

// dst = a*x + b*y (elementwise over [P][n])
template <typename T>
void axpby2d(int P, int n, double a, const T* x, int ldx, double b, const T* y,
             int ldy, T* dst, int ldd, hipStream_t st);
// the same with device coefficients: a = sa * ds[ia], b = sb * ds[ib] (an
// index < 0 takes sa or sb alone)
template <typename T>
void axpby2d_dev(int P, int n, double sa, int ia, const T* x, int ldx, double sb, int ib,
                 const T* y, int ldy, T* dst, int ldd, const double* ds, hipStream_t st);
// Interface PCG scalars in ds (device; sums over the P partials of a, b in
// a fixed order; P may count (row chunk, mode) partials):
// mode 0: ds[par] = sum a (r'z); mode 1: ds[2] = alpha = ds[par] / sum a
// (sum a = p'q; if not > 0: alpha = 0 and ds[4] = 1, or 2 if non-finite);
// mode 2: ds[3] = beta = (sum a - sum b) / ds[par], ds[1 - par] = sum a.
void outer_scalars(int mode, int P, const double* a, const double* b, double* ds, int par,
                   hipStream_t st);

// Newmark predictor (Eq. UmCm, UmCm2) and the mass-term vector of the force.
void newmark_predict(int P, int n, int ld, const double* U, const double* V,
                     const double* A, double dt, double zeta, double gamma,
                     double wc, double* Um, double* Uc, double* Wm,
                     hipStream_t st);
// Newmark update: A1 = U1/(zeta dt^2) - Um; V1 = V + dt((1-g)A + g A1)
void newmark_update(int P, int n, int ld, const double* U1, const double* Um,
                    double* V, double* A, double dt, double zeta, double gamma,
                    hipStream_t st);
// The same two steps with the images of the state under the SG operator K~
// carried along (both steps are linear, so K~ of each combination is the
// combination of GU = K~ U, GV = K~ V, GA = K~ A).  Predictor: Um and Wm as
// above, and F = c1 K~ Uc (the stiffness-damping share of the force).
// Update: V, A as above, and GU = F - R (K~ U1, with R = F - K~ U1 the
// final residual of the step's solve), GA, GV by the update's formulas.
void newmark_predict_g(int P, int ld, const double* U, const double* V, const double* A,
                       const double* GU, const double* GV, const double* GA, double dt,
                       double zeta, double gamma, double wc, double c1, double* Um, double* Wm,
                       double* F, hipStream_t st);
// R = F - (GU + cv GV + ca GA): the residual of X0 = U + cv V + ca A from the
// images of the state.
void residual_images(int P, int ld, const double* F, const double* GU, const double* GV,
                     const double* GA, double cv, double ca, double* R, hipStream_t st);
void newmark_update_g(int P, int ld, const double* U1, const double* Um, const double* F,
                      const double* R, double* V, double* A, double* GU, double* GV, double* GA,
                      double dt, double zeta, double gamma, hipStream_t st);

// Interface <-> torn maps (D_s R_s and sum_s R_s^T D_s) and the coarse grid.
template <typename T>
void scatter_to_torn(int NT, int P, const int* gidx, const double* w,
                     const T* r, int ldr, T* bt, int ldt, hipStream_t st);
template <typename T>
void gather_from_torn(int nG, int P, const int* gptr, const int* gtorn,
                      const double* gw, const int* g2c, const T* ut, int ldt,
                      const double* uc, int ldc, T* z, int ldz, hipStream_t st);
struct DCoarse {
  int nC = 0, P = 0, nk = 0, maxc = 0;
  const int *c_ptr, *c_lc;        // coarse index -> local corners
  const int *sc_gidx, *sc_coarse;  // local corner -> interface index, coarse index
  const double* sc_w;
  const int *cc_ptr, *cc_torn;     // local corner -> torn couplings
  const double* cc_val;            // [entry][nk]
  const int *gi_ptr, *gi_k, *gi_j; // Galerkin entries by output mode i
  const double* gi_v;
  const int *rem_off, *rem_list;   // remaining torn rows per subdomain
  const int* sc_ptr;               // local corners per subdomain
  const double* phi;               // coarse basis, per subdomain blocks
  const unsigned short* phih;      // its FP16 copy (bit patterns; FP32 solver only), each
                                   // subdomain's rows padded to a multiple of 4 values
  const long long* phi_off;
  const long long* phih_off;
  int max_rem = 0;                 // largest number of remaining rows
};
// local coarse unknowns (P x corners) of one subdomain held in LDS by the lift
#define SGW_MAX_COARSE_LOCAL 4096
template <typename T>
void coarse_rhs(const DCoarse& c, const T* r, int ldr, const T* yt, int ldt,
                double* dc, hipStream_t st);
// Factor of F_cc on the device (see coarse.h): R corner rows, row offsets
// off (host) in the factor's unknown order w, perm[w] = m * nC + corner of
// the coarse vectors; per row i the inverse diagonal block linv[i] and its
// transpose linvT[i] (m_i x m_i), per row i < R-1 the sub-diagonal block
// b[i] = L_{i+1,i} (m_{i+1} x m_i) and bT[i] = its transpose, all row-major;
// four work vectors of n; FP32 copies of the blocks for the FP32 solver
// (single = true: the same sweeps read them, accumulating in FP64).
struct DCoarseFactor {
  int R = 0, n = 0;
  std::vector<int> off;
  std::vector<const double*> linv, linvT, b, bT;
  std::vector<const float*> linvf, linvTf, bf, bTf;
  const int* perm = nullptr;
  double *wd = nullptr, *wy = nullptr, *wt = nullptr, *wx = nullptr;
};
void coarse_solve(const DCoarseFactor& f, const double* dc, double* uc, bool single,
                  hipStream_t st);
template <typename T>
void coarse_lift(const DCoarse& c, int nsub, const double* uc, T* ut, int ldt,
                 hipStream_t st);
// c.phih = FP16 (round to nearest, via FP32) copy of c.phi in its padded layout;
// nq[s], nout[s]: coarse unknowns and outputs of subdomain s (device arrays)
void coarse_basis_to_half(const DCoarse& c, int nsub, const int* nq, const long long* nout,
                          hipStream_t st);

}  // namespace k
}  // namespace sgw
