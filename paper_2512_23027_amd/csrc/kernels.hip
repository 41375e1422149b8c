// HIP kernels of the SG wave solver for gfx950 (CDNA4, wave64).
//
// Data layout: every SG vector is mode-major (one contiguous block of rows
// per PCE mode, Eq. GAssembly_Sto), sparse matrices are sliced ELL with the
// rows of one slot contiguous.  With one lane per matrix row, every global
// load of matrix values, column indices and vector entries is coalesced, and
// the Galerkin contraction over the PCE modes runs in registers and LDS of
// the lane that owns the row.
#include "kernels.h"
#include "k1_common.h"

#include <hip/hip_ext.h>

#include <algorithm>
#include <type_traits>
#include <cstdio>

namespace sgw {
namespace k {

#define SGW_WAVE 64
#define SGW_BLOCK 256
// triangular solves: threads per workgroup and rows per thread in the
// diagonal phase (levels may hold up to TRI_TPB * TRI_RPT rows)
#define TRI_TPB 1024
#define TRI_RPT 2
#define TRI_DPT 8   // inverse-block values per thread loaded ahead of the pull phase

static inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

template <typename T> __device__ __forceinline__ T fmadd(T a, T b, T c) { return fma(a, b, c); }

// ---------------------------------------------------------------------------
// K1: SG operator apply y_i = sum_k sum_j c_kij K_k x_j (Eq. stok / K_T_Sto).
// One wave = 64 consecutive rows, one lane per row.  The KC coefficient
// matrices of a chunk live in registers (7 values each); for every input mode
// j the lane loads its 7 neighbour values of x_j, forms
// W_kj = sum_s K_k[r,s] x_j[col_s] for the (k, j) pairs the Galerkin tensor
// needs, and scatters c_kij W_kj into the output modes of its group, held in
// LDS (one column per lane, no bank conflicts, no atomics).  The loops over
// j, k and the tensor entries are uniform across the wave; the tensor tables
// are read through the scalar cache.
// ---------------------------------------------------------------------------
template <typename T, int KC>
__global__ __launch_bounds__(SGW_WAVE) void k_sg_apply(
    DEll<T> A, GTab g, const T* __restrict__ entc, int r0, int nrows,
    const T* __restrict__ x, int ldx, T* __restrict__ y, int ldy, T alpha,
    T beta, long long sx, long long sy) {
  extern __shared__ unsigned char smem_raw[];
  T* yl = reinterpret_cast<T*>(smem_raw);
  const int lane = threadIdx.x;
  const int rl = blockIdx.x * SGW_WAVE + lane;
  const int grp = blockIdx.y;
  x += (long long)blockIdx.z * sx;
  y += (long long)blockIdx.z * sy;
  const bool live = rl < nrows;
  const int r = r0 + (live ? rl : nrows - 1);
  const int NR = A.nrows;
  int col[7];
#pragma unroll
  for (int s = 0; s < 7; ++s) col[s] = A.col[(size_t)s * NR + r];
  const int i0 = grp * g.GS;
  const int gsz = min(g.GS, g.P - i0);
  for (int i = 0; i < gsz; ++i) yl[i * SGW_WAVE + lane] = T(0);
  for (int ch = 0; ch < g.nch; ++ch) {
    T kr[KC][7];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const int kx = ch * KC + kk;
#pragma unroll
      for (int s = 0; s < 7; ++s)
        kr[kk][s] = kx < A.nk ? A.val[((size_t)kx * 7 + s) * NR + r] : T(0);
    }
    const int tb = (grp * g.nch + ch) * g.P;
    for (int j = 0; j < g.P; ++j) {
      const uint32_t m = g.mask[tb + j];
      if (!m) continue;
      const T* xj = x + (size_t)j * ldx;
      T u[7];
#pragma unroll
      for (int s = 0; s < 7; ++s) u[s] = xj[col[s]];
      int pp = g.pair_beg[tb + j];
      int e = g.ent_beg[tb + j];
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) {
        if (m & (1u << kk)) {
          T w = kr[kk][0] * u[0];
#pragma unroll
          for (int s = 1; s < 7; ++s) w = fmadd(kr[kk][s], u[s], w);
          const int cnt = g.pair_cnt[pp++];
          for (int t = 0; t < cnt; ++t) {
            T* dst = &yl[g.ent_i[e + t] * SGW_WAVE + lane];
            *dst = fmadd(entc[e + t], w, *dst);
          }
          e += cnt;
        }
      }
    }
  }
  if (live) {
    for (int i = 0; i < gsz; ++i) {
      T* yp = y + (size_t)(i0 + i) * ldy + r;
      T v = alpha * yl[i * SGW_WAVE + lane];
      if (beta != T(0)) v = fmadd(beta, *yp, v);
      *yp = v;
    }
  }
}

// Kernels with the Galerkin tensor of a fixed basis unrolled (gen_k1.py),
// compiled in their own translation units (k1_gen_*.hip).
#include "k1_dispatch.inc"

template <typename T>
void sg_apply(const DEll<T>& A, const GTab& g, const DHalo* H, int r0, int nrows, const T* x,
              int ldx, T* y, int ldy, T alpha, T beta, int nbatch,
              long long sx, long long sy, hipStream_t st) {
  if (nrows <= 0) return;
  // the generated kernel when the basis has one and its LDS fits the halo
  if (g.use_spec && H && halo_groups(*H, r0, nrows) > 0 &&
      sg_apply_specialised<T>(g.L, g.p_in, g.p_out, A, *H, r0, nrows, x, ldx, y, ldy, alpha,
                              beta, nbatch, sx, sy, st))
    return;
  dim3 grid(ceil_div(nrows, SGW_WAVE), g.ng, nbatch);
  size_t sh = (size_t)g.GS * SGW_WAVE * sizeof(T);
  const T* entc = nullptr;
  if constexpr (sizeof(T) == 8) entc = reinterpret_cast<const T*>(g.ent_c);
  else entc = reinterpret_cast<const T*>(g.ent_cf);
  switch (g.KC) {
    case 4:
      k_sg_apply<T, 4><<<grid, SGW_WAVE, sh, st>>>(A, g, entc, r0, nrows, x, ldx, y, ldy, alpha, beta, sx, sy);
      break;
    case 8:
      k_sg_apply<T, 8><<<grid, SGW_WAVE, sh, st>>>(A, g, entc, r0, nrows, x, ldx, y, ldy, alpha, beta, sx, sy);
      break;
    default:
      k_sg_apply<T, 16><<<grid, SGW_WAVE, sh, st>>>(A, g, entc, r0, nrows, x, ldx, y, ldy, alpha, beta, sx, sy);
      break;
  }
}

int sg_apply_prepare() { return sg_apply_specialised_prepare() ? 0 : -1; }
int sg_apply_generated(int L, int p_in, int p_out, int wbytes) {
  return sg_apply_specialised_groups(L, p_in, p_out, wbytes);
}

template <typename T>
bool sg_apply_pcg_fits(const GTab& g, const DHalo& H) {
  if (!g.use_spec || H.aligned64 || !H.bgrp) return false;
  const size_t lds = sg_apply_specialised_lds<T>(g.L, g.p_in, g.p_out, H.hmax, true);
  return lds > 0 && lds <= 160 * 1024;
}

template <typename T>
bool sg_apply_pcg(const DEll<T>& A, const GTab& g, const DHalo& H, int nrows, const T* pold,
                  const T* z, T* pnew, int ld, T* q, const double* rzpart, double* sc, int par,
                  double* pqg, unsigned long long* acct, unsigned bpr, hipStream_t st) {
  if (!sg_apply_pcg_fits<T>(g, H) || nrows != H.nr) return false;
  return sg_apply_pcg_specialised<T>(g.L, g.p_in, g.p_out, A, H, nrows, pold, z, pnew, ld, q,
                                     rzpart, sc, par, pqg, acct, bpr, st);
}

// Deterministic mass apply over all P modes: thread per (row, mode).
template <typename T>
__global__ void k_mass_apply(DEll<T> A, int r0, int nrows, int P, const T* __restrict__ x,
                             int ldx, T* __restrict__ y, int ldy, T alpha, T beta) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nrows * P) return;
  int j = (int)(t / nrows), r = r0 + (int)(t % nrows);
  const int NR = A.nrows;
  T s = T(0);
#pragma unroll
  for (int q = 0; q < 7; ++q)
    s = fmadd(A.mval[(size_t)q * NR + r], x[(size_t)j * ldx + A.col[(size_t)q * NR + r]], s);
  T* yp = y + (size_t)j * ldy + r;
  T v = alpha * s;
  if (beta != T(0)) v = fmadd(beta, *yp, v);
  *yp = v;
}

template <typename T>
void mass_apply(const DEll<T>& A, int r0, int nrows, int P, const T* x, int ldx,
                T* y, int ldy, T alpha, T beta, hipStream_t st) {
  long long n = (long long)nrows * P;
  if (n <= 0) return;
  k_mass_apply<T><<<ceil_div(n, SGW_BLOCK), SGW_BLOCK, 0, st>>>(A, r0, nrows, P, x, ldx, y, ldy, alpha, beta);
}

// ---------------------------------------------------------------------------
// K3: batched supernodal triangular solves with the mean-matrix factor
// L L^T = K~_0^s (the inner preconditioner I_P (x) K~_0^{-1}).  One workgroup
// per (subdomain block, tile of Q modes); the right-hand sides of the tile
// stay in LDS (row-major, Q values per row) for both sweeps.  Supernodes
// (nested-dissection sets) are processed level by level:
//  * pull phase, one thread per row, all Q modes in registers: the row takes
//    the contributions of the already-solved supernodes (forward: its
//    descendants through the rows of L; backward: its ancestors through the
//    columns of L);
//  * diagonal phase, one wave per supernode, one lane per row: the dense
//    inverse of the supernode's diagonal block is applied in place.  All
//    lanes of the wave read the block before any lane writes it, so no
//    workgroup barrier or scratch copy is needed.  The inverse is stored
//    column-major for the forward and row-major for the backward sweep, so
//    the lanes of a wave read it contiguously.
// Every sum has a fixed order: the result is bitwise reproducible.
// ---------------------------------------------------------------------------
template <typename T, int Q>
__global__ __launch_bounds__(TRI_TPB) void k_tri_solve(
    DFactor f, const T* __restrict__ lrv, const T* __restrict__ lcv,
    const T* __restrict__ dr, const T* __restrict__ dc, const T* rhs, int ldr,
    T* out, int ldo, long long sr, long long so) {
  extern __shared__ unsigned char smem_raw[];
  // LDS: right-hand sides; the dense inverse blocks of the current level;
  // the block's level lists, entry pointers and supernode table, so that
  // every index the sweeps need is one LDS read
  T* X = reinterpret_cast<T*>(smem_raw);
  T* Dst = X + (size_t)f.max_rows * Q;
  int* s_row = reinterpret_cast<int*>(Dst + f.max_lvl_d);
  int* s_sn = s_row + f.max_rows;
  int* s_lr = s_sn + f.max_rows;
  int* s_lc = s_lr + f.max_rows + 1;
  int* s_beg = s_lc + f.max_rows + 1;
  int* s_w = s_beg + f.max_sn;
  int* s_dv = s_w + f.max_sn;
  int* s_lrow = s_dv + f.max_sn;             // level -> first position
  int* s_lsn = s_lrow + f.max_levels + 1;     // level -> first supernode
  int* s_gf = s_lsn + f.max_levels + 1;
  int* s_gb = s_gf + f.max_levels + 1;
  const int b = f.order ? f.order[blockIdx.x] : blockIdx.x;  // largest blocks first
  const int q0 = blockIdx.y * Q;
  rhs += (long long)blockIdx.z * sr;
  out += (long long)blockIdx.z * so;
  const int r0 = f.row_off[b];
  const int n = f.row_off[b + 1] - r0;
  const int nq = min(Q, f.P - q0);
  const int tid = threadIdx.x;
  const int lo = f.lvl_off[b];
  const int nlev = f.lvl_off[b + 1] - lo - 1;
  const int p0 = f.lrow_ptr[lo];
  const int sn0 = f.lvl_ptr[lo];
  const int nsn = f.lvl_ptr[lo + nlev] - sn0;
  for (int i = tid; i < n; i += TRI_TPB) {
    s_row[i] = f.lrow_list[p0 + i];
    s_sn[i] = f.lrow_sn[p0 + i] - sn0;
  }
  for (int i = tid; i <= n; i += TRI_TPB) {
    s_lr[i] = f.lr_ptr[p0 + i];
    s_lc[i] = f.lc_ptr[p0 + i];
  }
  for (int i = tid; i < nsn; i += TRI_TPB) {
    s_beg[i] = f.sn_beg[sn0 + i];
    s_w[i] = f.sn_w[sn0 + i];
    s_dv[i] = f.sn_dinv[sn0 + i];
  }
  for (int i = tid; i <= nlev; i += TRI_TPB) {
    s_lrow[i] = f.lrow_ptr[lo + i] - p0;
    s_lsn[i] = f.lvl_ptr[lo + i] - sn0;
    s_gf[i] = f.lvl_gf[lo + i];
    s_gb[i] = f.lvl_gb[lo + i];
  }
  // coalesced load: consecutive threads take consecutive rows of one mode
  for (int idx = tid; idx < n * Q; idx += TRI_TPB) {
    int q = idx / n, r = idx - q * n;
    X[r * Q + q] = q < nq ? rhs[(size_t)(q0 + q) * ldr + r0 + r] : T(0);
  }
  __syncthreads();
  for (int sweep = 0; sweep < 2; ++sweep) {
    const bool fwd = sweep == 0;
    const int* sp = fwd ? s_lr : s_lc;
    const int* eidx = fwd ? f.lr_col : f.lc_row;
    const T* eval = fwd ? lrv : lcv;
    const T* dmat = fwd ? dc : dr;
    const int* sg = fwd ? s_gf : s_gb;
    for (int it = 0; it < nlev; ++it) {
      const int l = fwd ? nlev - 1 - it : it;
      const int ra = s_lrow[l], nr = s_lrow[l + 1] - ra;
      const int snA = s_lsn[l], snB = s_lsn[l + 1];
      // the inverse blocks of this level are contiguous: start their loads
      // now, store them to LDS after the pull phase
      const int d0 = snA < snB ? s_dv[snA] : 0;
      const int nd = snA < snB ? s_dv[snB - 1] + s_w[snB - 1] * s_w[snB - 1] - d0 : 0;
      T dreg[TRI_DPT];
#pragma unroll
      for (int t = 0; t < TRI_DPT; ++t) {
        const int j = tid + t * TRI_TPB;
        dreg[t] = j < nd ? dmat[(size_t)d0 + j] : T(0);
      }
      // pull phase: G consecutive lanes share one row (G divides 64); each
      // lane reads up to 8 of its entries at once, then a fixed xor-shuffle
      // tree adds the G partial sums
      const int G = sg[l];
      if (G > 0) {
        for (int idx = tid; idx < nr * G; idx += TRI_TPB) {
          const int li = ra + idx / G, sub = idx & (G - 1);
          const int row = s_row[li];
          const int e1 = sp[li + 1];
          T acc[Q];
#pragma unroll
          for (int q = 0; q < Q; ++q) acc[q] = T(0);
          for (int e = sp[li] + sub; e < e1; e += 8 * G) {
            int ci[8];
            T cv[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
              const int ee = e + t * G;
              const bool ok = ee < e1;
              ci[t] = ok ? eidx[ee] * Q : 0;
              cv[t] = ok ? eval[ee] : T(0);
            }
#pragma unroll
            for (int t = 0; t < 8; ++t)
#pragma unroll
              for (int q = 0; q < Q; ++q) acc[q] = fmadd(cv[t], X[ci[t] + q], acc[q]);
          }
          for (int off = G >> 1; off > 0; off >>= 1)
#pragma unroll
            for (int q = 0; q < Q; ++q) acc[q] += __shfl_xor(acc[q], off, 64);
          if (sub == 0)
#pragma unroll
            for (int q = 0; q < Q; ++q) X[row * Q + q] -= acc[q];
        }
      }
#pragma unroll
      for (int t = 0; t < TRI_DPT; ++t) {
        const int j = tid + t * TRI_TPB;
        if (j < nd) Dst[j] = dreg[t];
      }
      for (int j = tid + TRI_DPT * TRI_TPB; j < nd; j += TRI_TPB) Dst[j] = dmat[(size_t)d0 + j];
      __syncthreads();
      // diagonal phase: one thread per row of the level (at most TRI_RPT
      // rows per thread) applies its row of the supernode's dense inverse
      // from LDS; results wait in registers until every thread has read the
      // level's rows, then overwrite them
      T res[TRI_RPT][Q];
#pragma unroll
      for (int k2 = 0; k2 < TRI_RPT; ++k2) {
        const int idx = tid + k2 * TRI_TPB;
        if (idx < nr) {
          const int li = ra + idx, row = s_row[li], sn = s_sn[li];
          const int beg = s_beg[sn], w = s_w[sn], a = row - beg;
          const T* D = Dst + (s_dv[sn] - d0);
          T acc[Q];
#pragma unroll
          for (int q = 0; q < Q; ++q) acc[q] = T(0);
          for (int c = 0; c < w; ++c) {
            const T dv = D[c * w + a];
#pragma unroll
            for (int q = 0; q < Q; ++q) acc[q] = fmadd(dv, X[(beg + c) * Q + q], acc[q]);
          }
#pragma unroll
          for (int q = 0; q < Q; ++q) res[k2][q] = acc[q];
        }
      }
      __syncthreads();
#pragma unroll
      for (int k2 = 0; k2 < TRI_RPT; ++k2) {
        const int idx = tid + k2 * TRI_TPB;
        if (idx < nr) {
          const int row = s_row[ra + idx];
#pragma unroll
          for (int q = 0; q < Q; ++q) X[row * Q + q] = res[k2][q];
        }
      }
      __syncthreads();
    }
  }
  // coalesced store
  for (int idx = tid; idx < n * Q; idx += TRI_TPB) {
    int q = idx / n, r = idx - q * n;
    if (q < nq) out[(size_t)(q0 + q) * ldo + r0 + r] = X[r * Q + q];
  }
}

// LDS bytes of one triangular-solve workgroup with Q modes
template <typename T>
size_t tri_lds_bytes(const DFactor& f, int Q) {
  return ((size_t)f.max_rows * Q + (size_t)f.max_lvl_d) * sizeof(T) +
         sizeof(int) * (4 * (size_t)f.max_rows + 2 + 3 * (size_t)f.max_sn + 4 * ((size_t)f.max_levels + 1));
}

template <typename T, int Q>
static void launch_tri(const DFactor& f, const T* rhs, int ldr, T* out, int ldo,
                       int nbatch, long long sr, long long so, hipStream_t st) {
  size_t sh = tri_lds_bytes<T>(f, Q);
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)k_tri_solve<T, Q>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
  const T *lrv, *lcv, *dr, *dc;
  if constexpr (sizeof(T) == 8) {
    lrv = reinterpret_cast<const T*>(f.lr_val);
    lcv = reinterpret_cast<const T*>(f.lc_val);
    dr = reinterpret_cast<const T*>(f.dinv);
    dc = reinterpret_cast<const T*>(f.dinvT);
  } else {
    lrv = reinterpret_cast<const T*>(f.lr_valf);
    lcv = reinterpret_cast<const T*>(f.lc_valf);
    dr = reinterpret_cast<const T*>(f.dinvf);
    dc = reinterpret_cast<const T*>(f.dinvTf);
  }
  dim3 grid(f.nb, ceil_div(f.P, Q), nbatch);
  k_tri_solve<T, Q><<<grid, TRI_TPB, sh, st>>>(f, lrv, lcv, dr, dc, rhs, ldr, out, ldo, sr, so);
}

template <typename T>
void tri_solve(const DFactor& f, int Q, const T* rhs, int ldr, T* out, int ldo,
               int nbatch, long long sr, long long so, hipStream_t st) {
  switch (Q) {
    case 1: launch_tri<T, 1>(f, rhs, ldr, out, ldo, nbatch, sr, so, st); break;
    case 2: launch_tri<T, 2>(f, rhs, ldr, out, ldo, nbatch, sr, so, st); break;
    case 3: launch_tri<T, 3>(f, rhs, ldr, out, ldo, nbatch, sr, so, st); break;
    case 4: launch_tri<T, 4>(f, rhs, ldr, out, ldo, nbatch, sr, so, st); break;
    case 5: launch_tri<T, 5>(f, rhs, ldr, out, ldo, nbatch, sr, so, st); break;
    case 6: launch_tri<T, 6>(f, rhs, ldr, out, ldo, nbatch, sr, so, st); break;
    case 7: launch_tri<T, 7>(f, rhs, ldr, out, ldo, nbatch, sr, so, st); break;
    default: launch_tri<T, 8>(f, rhs, ldr, out, ldo, nbatch, sr, so, st); break;
  }
}

// ---------------------------------------------------------------------------
// K4: segmented reductions, FP64 accumulation, fixed order (wave shuffles
// then LDS), one workgroup per (block, mode).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += sh[q];
  return s;
}

template <typename T>
__global__ __launch_bounds__(SGW_BLOCK) void k_seg_dot(
    const int* row_off, int P, const T* a, int lda, const T* b, int ldb,
    double* part, const T* c, int ldc, const T* d, int ldd, double* part2) {
  __shared__ double sh[SGW_BLOCK / 64];
  const int blk = blockIdx.x, j = blockIdx.y;
  const int r0 = row_off[blk], r1 = row_off[blk + 1];
  double s = 0.0, s2 = 0.0;
  const T* ap = a + (size_t)j * lda;
  const T* bp = b + (size_t)j * ldb;
  for (int r = r0 + threadIdx.x; r < r1; r += SGW_BLOCK) s += (double)ap[r] * (double)bp[r];
  if (part2) {
    const T* cp = c + (size_t)j * ldc;
    const T* dp = d + (size_t)j * ldd;
    for (int r = r0 + threadIdx.x; r < r1; r += SGW_BLOCK) s2 += (double)cp[r] * (double)dp[r];
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blk * P + j] = s;
  if (part2) {
    s2 = block_sum(s2, sh);
    if (threadIdx.x == 0) part2[blk * P + j] = s2;
  }
}

template <typename T>
void seg_dot(int nb, const int* row_off, int P, const T* a, int lda, const T* b,
             int ldb, double* partial, const T* c, int ldc, const T* d, int ldd,
             double* partial2, hipStream_t st) {
  k_seg_dot<T><<<dim3(nb, P), SGW_BLOCK, 0, st>>>(row_off, P, a, lda, b, ldb, partial, c, ldc, d, ldd, partial2);
}

// ---------------------------------------------------------------------------
// Batched block PCG bookkeeping.  Every block b of the batch runs its own PCG
// (own step lengths, own stopping test); the per-block scalars live in
// sc[b*8 + ...]:
//   0, 1  r'z of iterations with even / odd index (parity slots)
//   2, 3  active flag (1.0 / 0.0) of even / odd iterations
//   4     b'b (squared norm of the right-hand side)
// Iteration `it` (parity p = it & 1) reads the p slots and writes the 1-p
// slots, so the workgroups of one block that read a scalar never race with
// the one that writes its successor.  Partial sums over (block, mode) come
// from the vector kernels: part = p'q, then r'z; part2 = r'r.
// flags[0] = number of active blocks after the last test, flags[1] |=
// breakdown (p'q <= 0 on an active block), flags[2] |= non-finite value.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_max(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double m = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) m = fmax(m, sh[q]);
  return m;
}

// Sum of p[0..n) in index order.  The loads of a chunk are issued together,
// so a sum costs one memory round trip per chunk instead of one per value.
__device__ __forceinline__ double sum_seq(const double* p, int n) {
  double v = 0.0;
  int j = 0;
  for (; j + 16 <= n; j += 16) {
    double t[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) t[k] = p[j + k];
#pragma unroll
    for (int k = 0; k < 16; ++k) v += t[k];
  }
  if (j + 4 <= n) {
    double t[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) t[k] = p[j + k];
#pragma unroll
    for (int k = 0; k < 4; ++k) v += t[k];
    j += 4;
  }
  for (; j < n; ++j) v += p[j];
  return v;
}

// the P partials of block b, in mode order
__device__ __forceinline__ double sum_modes(const double* part, int b, int P) {
  return sum_seq(part + (size_t)b * P, P);
}

// Start of a solve (x0 = 0, r = b, z = M r): r'z into the even slot, b'b = r'r,
// active = b'b > negl * max_b b'b and r'r > tol2 b'b.  A block whose
// right-hand side is negligible within the batch (negl > 0) keeps x = 0 -- in
// FP32 such blocks would underflow.  One workgroup for all blocks.
__global__ __launch_bounds__(SGW_BLOCK) void k_pcg_start(int nb, int P, const double* part,
                                                        const double* part2, double* sc,
                                                        double tol2, double negl, int* flags) {
  __shared__ int nact, bad;
  __shared__ double shm[SGW_BLOCK / 64];
  if (threadIdx.x == 0) {
    nact = 0;
    bad = 0;
  }
  __syncthreads();
  double m = 0.0;
  for (int b = threadIdx.x; b < nb; b += SGW_BLOCK) {
    const double rz = sum_modes(part, b, P), rr = sum_modes(part2, b, P);
    double* s = sc + (size_t)b * 8;
    s[0] = rz;
    s[4] = rr;
    if (!isfinite(rz) || !isfinite(rr)) atomicOr(&bad, 1);
    if (isfinite(rr)) m = fmax(m, rr);
  }
  const double floor_bb = negl * block_max(m, shm);
  for (int b = threadIdx.x; b < nb; b += SGW_BLOCK) {
    double* s = sc + (size_t)b * 8;
    const bool act = s[4] > floor_bb && s[4] > tol2 * s[4] && s[4] > 0.0;
    s[2] = act ? 1.0 : 0.0;
    s[1] = INFINITY;  // "previous r'z" of iteration 0: beta = 0 in the fused SG apply
    s[5] = 0.0;       // iterations taken by the block
    if (act) atomicAdd(&nact, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    flags[0] = nact;
    flags[1] = 0;
    flags[2] = bad;
    flags[3] = 0;
  }
}

void pcg_start(int nb, int P, const double* part, const double* part2, double* sc, double tol2,
               double negl, int* flags, hipStream_t st) {
  k_pcg_start<<<1, SGW_BLOCK, 0, st>>>(nb, P, part, part2, sc, tol2, negl, flags);
}

// x += alpha p, r -= alpha q on the active blocks, alpha = r'z / p'q of the
// block (p'q summed from part); writes part2 = r'r per (block, mode) of the
// active blocks (a converged block is frozen: its r'r is not read again).
// Counts the block's iterations in sc[8b + 5] and keeps their maximum over
// the blocks in flags[3].  Workgroup (0, 0) clears the active counter for the
// test that follows.  A workgroup takes XR_MODES modes of one block (the
// loads of a row's modes are independent and in flight together).
#define XR_MODES 4
template <typename T>
__global__ __launch_bounds__(SGW_BLOCK) void k_pcg_xr(
    const int* row_off, int P, int par, double* sc, T* __restrict__ x, int ldx,
    const T* __restrict__ p, int ldp, T* __restrict__ r, int ldr, const T* __restrict__ q,
    int ldq, const double* part, double* part2, int* flags, const int* bgrp, int pqn) {
  __shared__ double sh[SGW_BLOCK / 64][XR_MODES];
  const int blk = blockIdx.x, j0 = blockIdx.y * XR_MODES;
  const int r0 = row_off[blk], r1 = row_off[blk + 1];
  double* s = sc + (size_t)blk * 8;
  const bool act = s[2 + par] != 0.0;
  if (blk == 0 && blockIdx.y == 0 && threadIdx.x == 0) flags[0] = 0;
  if (!act) return;
  if (blockIdx.y == 0 && threadIdx.x == 0) {
    s[5] += 1.0;
    atomicMax(&flags[3], (int)s[5]);
  }
  double al = 0.0;
  {
    double pq = 0.0;
    if (bgrp) {  // per-group partials of the fused SG apply (pqn per group)
      pq = sum_seq(part + (size_t)bgrp[blk] * pqn, (bgrp[blk + 1] - bgrp[blk]) * pqn);
    } else {
      pq = sum_modes(part, blk, P);
    }
    if (pq > 0.0) {
      al = s[par] / pq;
    } else if (blockIdx.y == 0 && threadIdx.x == 0) {
      if (isfinite(pq)) atomicOr(&flags[1], 1);
      else atomicOr(&flags[2], 1);
    }
  }
  const T alt = (T)al;
  const int nq = min(XR_MODES, P - j0);
  double acc[XR_MODES];
#pragma unroll
  for (int m = 0; m < XR_MODES; ++m) acc[m] = 0.0;
  // modes past P repeat the last one (loaded, not stored or counted)
  size_t jo[XR_MODES];
#pragma unroll
  for (int m = 0; m < XR_MODES; ++m) jo[m] = (size_t)(j0 + min(m, nq - 1));
  for (int i = r0 + threadIdx.x; i < r1; i += SGW_BLOCK) {
    T rv[XR_MODES], xv[XR_MODES], pv[XR_MODES], qv[XR_MODES];
#pragma unroll
    for (int m = 0; m < XR_MODES; ++m) {
      rv[m] = r[jo[m] * ldr + i];
      xv[m] = x[jo[m] * ldx + i];
      pv[m] = p[jo[m] * ldp + i];
      qv[m] = q[jo[m] * ldq + i];
    }
#pragma unroll
    for (int m = 0; m < XR_MODES; ++m) {
      if (m >= nq) break;
      if (al != 0.0) {
        x[jo[m] * ldx + i] = fmadd(alt, pv[m], xv[m]);
        rv[m] = fmadd(-alt, qv[m], rv[m]);
        r[jo[m] * ldr + i] = rv[m];
      }
      acc[m] += (double)rv[m] * (double)rv[m];
    }
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int m = 0; m < XR_MODES; ++m) {
    const double v = wave_sum(acc[m]);
    if (lane == 0) sh[w][m] = v;
  }
  __syncthreads();
  if (threadIdx.x < nq) {
    double t = 0.0;
    for (int v = 0; v < SGW_BLOCK / 64; ++v) t += sh[v][threadIdx.x];
    part2[(size_t)blk * P + j0 + threadIdx.x] = t;
  }
}

template <typename T>
void pcg_xr(int nb, const int* row_off, int P, int par, double* sc, T* x, int ldx,
            const T* p, int ldp, T* r, int ldr, const T* q, int ldq, const double* part,
            double* part2, int* flags, hipStream_t st, const int* bgrp, int pqn) {
  k_pcg_xr<T><<<dim3(nb, ceil_div(P, XR_MODES)), SGW_BLOCK, 0, st>>>(
      row_off, P, par, sc, x, ldx, p, ldp, r, ldr, q, ldq, part, part2, flags, bgrp, pqn);
}

// Stopping test of iteration par (used with the exact preconditioner; the
// Chebyshev kernel does the same test itself): active' = active and
// r'r > tol2 b'b, written to the other parity slot and counted in flags[0].
__global__ __launch_bounds__(SGW_BLOCK) void k_pcg_test(int nb, int P, int par,
                                                       const double* part2, double* sc,
                                                       double tol2, int* flags) {
  __shared__ int nact, bad;
  if (threadIdx.x == 0) {
    nact = 0;
    bad = 0;
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += SGW_BLOCK) {
    double* s = sc + (size_t)b * 8;
    const double rr = sum_modes(part2, b, P);
    if (!isfinite(rr)) atomicOr(&bad, 1);
    const bool act = s[2 + par] != 0.0 && rr > tol2 * s[4];
    s[3 - par] = act ? 1.0 : 0.0;
    if (act) atomicAdd(&nact, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    flags[0] = nact;
    if (bad) flags[2] = 1;
  }
}

void pcg_test(int nb, int P, int par, const double* part2, double* sc, double tol2, int* flags,
              hipStream_t st) {
  k_pcg_test<<<1, SGW_BLOCK, 0, st>>>(nb, P, par, part2, sc, tol2, flags);
}

// p = z + beta p on the blocks still active after the test of iteration par,
// beta = (new r'z from part) / (old r'z); workgroup (b, 0) stores the new r'z
// in the other parity slot.
template <typename T>
__global__ __launch_bounds__(SGW_BLOCK) void k_pcg_p(const int* row_off, int P, int par,
                                                    double* sc, const double* part, const T* z,
                                                    int ldz, T* p, int ldp) {
  const int blk = blockIdx.x, j = blockIdx.y;
  double* s = sc + (size_t)blk * 8;
  if (s[3 - par] == 0.0) return;
  const double rz = sum_modes(part, blk, P);
  const T be = (T)(rz / s[par]);
  if (j == 0 && threadIdx.x == 0) s[1 - par] = rz;
  const int r0 = row_off[blk], r1 = row_off[blk + 1];
  const T* zp = z + (size_t)j * ldz;
  T* pp = p + (size_t)j * ldp;
  for (int i = r0 + threadIdx.x; i < r1; i += SGW_BLOCK) pp[i] = fmadd(be, pp[i], zp[i]);
}

template <typename T>
void pcg_p(int nb, const int* row_off, int P, int par, double* sc, const double* part,
           const T* z, int ldz, T* p, int ldp, hipStream_t st) {
  k_pcg_p<T><<<dim3(nb, P), SGW_BLOCK, 0, st>>>(row_off, P, par, sc, part, z, ldz, p, ldp);
}


// ---------------------------------------------------------------------------
// Elementwise helpers over mode-major [P][n] arrays.
// ---------------------------------------------------------------------------
template <typename TD, typename TS>
__global__ void k_copy2d(int P, int n, const TS* src, int lds, TD* dst, int ldd, double a) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)P * n) return;
  int j = (int)(t / n), r = (int)(t % n);
  dst[(size_t)j * ldd + r] = (TD)(a * (double)src[(size_t)j * lds + r]);
}
template <typename TD, typename TS>
void copy2d(int P, int n, const TS* src, int lds, TD* dst, int ldd, double a, hipStream_t st) {
  long long N = (long long)P * n;
  if (N > 0) k_copy2d<TD, TS><<<ceil_div(N, SGW_BLOCK), SGW_BLOCK, 0, st>>>(P, n, src, lds, dst, ldd, a);
}

template <typename T>
__global__ void k_fill2d(int P, int n, T* dst, int ldd, T v) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)P * n) return;
  int j = (int)(t / n), r = (int)(t % n);
  dst[(size_t)j * ldd + r] = v;
}
template <typename T>
void fill2d(int P, int n, T* dst, int ldd, T v, hipStream_t st) {
  long long N = (long long)P * n;
  if (N > 0) k_fill2d<T><<<ceil_div(N, SGW_BLOCK), SGW_BLOCK, 0, st>>>(P, n, dst, ldd, v);
}

template <typename T>
__global__ void k_axpby2d(int P, int n, double a, const T* x, int ldx, double b,
                          const T* y, int ldy, T* dst, int ldd) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)P * n) return;
  int j = (int)(t / n), r = (int)(t % n);
  double v = a * (double)x[(size_t)j * ldx + r] + b * (double)y[(size_t)j * ldy + r];
  dst[(size_t)j * ldd + r] = (T)v;
}
template <typename T>
void axpby2d(int P, int n, double a, const T* x, int ldx, double b, const T* y,
             int ldy, T* dst, int ldd, hipStream_t st) {
  long long N = (long long)P * n;
  if (N > 0) k_axpby2d<T><<<ceil_div(N, SGW_BLOCK), SGW_BLOCK, 0, st>>>(P, n, a, x, ldx, b, y, ldy, dst, ldd);
}

// dst = sa * (ia >= 0 ? ds[ia] : 1) * x + sb * (ib >= 0 ? ds[ib] : 1) * y with
// the coefficients read from device scalars
template <typename T>
__global__ void k_axpby2d_dev(int P, int n, double sa, int ia, const T* x, int ldx, double sb,
                              int ib, const T* y, int ldy, T* dst, int ldd, const double* ds) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)P * n) return;
  const double a = ia >= 0 ? sa * ds[ia] : sa, b = ib >= 0 ? sb * ds[ib] : sb;
  int j = (int)(t / n), r = (int)(t % n);
  double v = a * (double)x[(size_t)j * ldx + r] + b * (double)y[(size_t)j * ldy + r];
  dst[(size_t)j * ldd + r] = (T)v;
}
template <typename T>
void axpby2d_dev(int P, int n, double sa, int ia, const T* x, int ldx, double sb, int ib,
                 const T* y, int ldy, T* dst, int ldd, const double* ds, hipStream_t st) {
  long long N = (long long)P * n;
  if (N > 0)
    k_axpby2d_dev<T><<<ceil_div(N, SGW_BLOCK), SGW_BLOCK, 0, st>>>(P, n, sa, ia, x, ldx, sb, ib,
                                                                   y, ldy, dst, ldd, ds);
}

// Scalars of the interface PCG (one workgroup; the partial sums are added
// in a fixed order: per thread over a stride, then the threads' sums)
__global__ __launch_bounds__(SGW_BLOCK) void k_outer_scalars(int mode, int P, const double* a,
                                                            const double* b, double* ds,
                                                            int par) {
  __shared__ double sh[SGW_BLOCK / 64];
  double va = 0.0, vb = 0.0;
  for (int j = threadIdx.x; j < P; j += SGW_BLOCK) {
    va += a[j];
    if (mode == 2) vb += b[j];
  }
  const double sa = block_sum(va, sh);
  const double sb = mode == 2 ? block_sum(vb, sh) : 0.0;
  if (threadIdx.x != 0) return;
  if (mode == 0) {  // start: r'z
    ds[par] = sa;
  } else if (mode == 1) {  // alpha = r'z / p'q, breakdown flag
    if (sa > 0.0) {
      ds[2] = ds[par] / sa;
    } else {
      ds[2] = 0.0;
      ds[4] = isfinite(sa) ? 1.0 : 2.0;
    }
  } else {  // flexible beta = (r'z - r'z_prev) / r'z_old; r'z of the next iteration
    ds[3] = (sa - sb) / ds[par];
    ds[1 - par] = sa;
  }
}
void outer_scalars(int mode, int P, const double* a, const double* b, double* ds, int par,
                   hipStream_t st) {
  k_outer_scalars<<<1, SGW_BLOCK, 0, st>>>(mode, P, a, b, ds, par);
}

// ---------------------------------------------------------------------------
// K7: Newmark predictor (Eq. UmCm, UmCm2) and update (Sec. 2).
// Wm = Um + wc Uc is the vector the mass matrix multiplies in the effective
// force (Eq. fparts with Rayleigh damping).
// ---------------------------------------------------------------------------
__global__ void k_newmark_predict(long long N, const double* U, const double* V,
                                  const double* A, double dt, double zeta, double gamma,
                                  double wc, double* Um, double* Uc, double* Wm) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  double um = (U[t] + dt * V[t]) / (zeta * dt * dt) + (1.0 - 2.0 * zeta) * A[t] / (2.0 * zeta);
  double uc = gamma * dt * um - V[t] - (1.0 - gamma) * dt * A[t];
  Um[t] = um;
  Uc[t] = uc;
  Wm[t] = um + wc * uc;
}
void newmark_predict(int P, int n, int ld, const double* U, const double* V,
                     const double* A, double dt, double zeta, double gamma, double wc,
                     double* Um, double* Uc, double* Wm, hipStream_t st) {
  long long N = (long long)P * ld;
  (void)n;
  k_newmark_predict<<<ceil_div(N, SGW_BLOCK), SGW_BLOCK, 0, st>>>(N, U, V, A, dt, zeta, gamma, wc, Um, Uc, Wm);
}

__global__ void k_newmark_update(long long N, const double* U1, const double* Um,
                                 double* V, double* A, double dt, double zeta, double gamma) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  double a1 = U1[t] / (zeta * dt * dt) - Um[t];
  V[t] = V[t] + dt * ((1.0 - gamma) * A[t] + gamma * a1);
  A[t] = a1;
}
void newmark_update(int P, int n, int ld, const double* U1, const double* Um, double* V,
                    double* A, double dt, double zeta, double gamma, hipStream_t st) {
  long long N = (long long)P * ld;
  (void)n;
  k_newmark_update<<<ceil_div(N, SGW_BLOCK), SGW_BLOCK, 0, st>>>(N, U1, Um, V, A, dt, zeta, gamma);
}

__global__ void k_newmark_predict_g(long long N, const double* U, const double* V,
                                    const double* A, const double* GU, const double* GV,
                                    const double* GA, double dt, double zeta, double gamma,
                                    double wc, double c1, double* Um, double* Wm, double* F) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const double um = (U[t] + dt * V[t]) / (zeta * dt * dt) + (1.0 - 2.0 * zeta) * A[t] / (2.0 * zeta);
  const double uc = gamma * dt * um - V[t] - (1.0 - gamma) * dt * A[t];
  const double gum =
      (GU[t] + dt * GV[t]) / (zeta * dt * dt) + (1.0 - 2.0 * zeta) * GA[t] / (2.0 * zeta);
  const double guc = gamma * dt * gum - GV[t] - (1.0 - gamma) * dt * GA[t];
  Um[t] = um;
  Wm[t] = um + wc * uc;
  F[t] = c1 * guc;
}
void newmark_predict_g(int P, int ld, const double* U, const double* V, const double* A,
                       const double* GU, const double* GV, const double* GA, double dt,
                       double zeta, double gamma, double wc, double c1, double* Um, double* Wm,
                       double* F, hipStream_t st) {
  long long N = (long long)P * ld;
  k_newmark_predict_g<<<ceil_div(N, SGW_BLOCK), SGW_BLOCK, 0, st>>>(N, U, V, A, GU, GV, GA, dt,
                                                                     zeta, gamma, wc, c1, Um, Wm,
                                                                     F);
}

__global__ void k_residual_images(long long N, const double* F, const double* GU,
                                  const double* GV, const double* GA, double cv, double ca,
                                  double* R) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  R[t] = F[t] - ((GU[t] + cv * GV[t]) + ca * GA[t]);
}
void residual_images(int P, int ld, const double* F, const double* GU, const double* GV,
                     const double* GA, double cv, double ca, double* R, hipStream_t st) {
  long long N = (long long)P * ld;
  k_residual_images<<<ceil_div(N, SGW_BLOCK), SGW_BLOCK, 0, st>>>(N, F, GU, GV, GA, cv, ca, R);
}

__global__ void k_newmark_update_g(long long N, const double* U1, const double* Um,
                                   const double* F, const double* R, double* V, double* A,
                                   double* GU, double* GV, double* GA, double dt, double zeta,
                                   double gamma) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const double a1 = U1[t] / (zeta * dt * dt) - Um[t];
  V[t] = V[t] + dt * ((1.0 - gamma) * A[t] + gamma * a1);
  A[t] = a1;
  // K~ Um from the images of the old state, as in the predictor
  const double gum =
      (GU[t] + dt * GV[t]) / (zeta * dt * dt) + (1.0 - 2.0 * zeta) * GA[t] / (2.0 * zeta);
  const double gu1 = F[t] - R[t];
  const double ga1 = gu1 / (zeta * dt * dt) - gum;
  GV[t] = GV[t] + dt * ((1.0 - gamma) * GA[t] + gamma * ga1);
  GA[t] = ga1;
  GU[t] = gu1;
}
void newmark_update_g(int P, int ld, const double* U1, const double* Um, const double* F,
                      const double* R, double* V, double* A, double* GU, double* GV, double* GA,
                      double dt, double zeta, double gamma, hipStream_t st) {
  long long N = (long long)P * ld;
  k_newmark_update_g<<<ceil_div(N, SGW_BLOCK), SGW_BLOCK, 0, st>>>(N, U1, Um, F, R, V, A, GU, GV,
                                                                    GA, dt, zeta, gamma);
}

// ---------------------------------------------------------------------------
// K6: interface restriction with partition-of-unity weights (D_s R_s,
// Eq. det_scaling) into the torn Neumann vectors, and the weighted
// owner-computes gather sum_s R_s^T D_s back to the interface (Eq. ugb).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_scatter_to_torn(int NT, int P, const int* gidx, const double* w,
                                  const T* r, int ldr, T* bt, int ldt) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)NT * P) return;
  int j = (int)(t / NT), row = (int)(t % NT);
  int g = gidx[row];
  bt[(size_t)j * ldt + row] = g >= 0 ? (T)(w[row] * (double)r[(size_t)j * ldr + g]) : T(0);
}
template <typename T>
void scatter_to_torn(int NT, int P, const int* gidx, const double* w, const T* r,
                     int ldr, T* bt, int ldt, hipStream_t st) {
  long long N = (long long)NT * P;
  k_scatter_to_torn<T><<<ceil_div(N, SGW_BLOCK), SGW_BLOCK, 0, st>>>(NT, P, gidx, w, r, ldr, bt, ldt);
}

template <typename T>
__global__ void k_gather_from_torn(int nG, int P, const int* gptr, const int* gtorn,
                                   const double* gw, const int* g2c, const T* ut, int ldt,
                                   const double* uc, int ldc, T* z, int ldz) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nG * P) return;
  int j = (int)(t / nG), g = (int)(t % nG);
  double s = 0.0;
  int c = g2c[g];
  if (c >= 0) {
    s = (double)uc[(size_t)j * ldc + c];
  } else {
    for (int e = gptr[g]; e < gptr[g + 1]; ++e) s += gw[e] * (double)ut[(size_t)j * ldt + gtorn[e]];
  }
  z[(size_t)j * ldz + g] = (T)s;
}
template <typename T>
void gather_from_torn(int nG, int P, const int* gptr, const int* gtorn, const double* gw,
                      const int* g2c, const T* ut, int ldt, const double* uc, int ldc, T* z,
                      int ldz, hipStream_t st) {
  long long N = (long long)nG * P;
  k_gather_from_torn<T><<<ceil_div(N, SGW_BLOCK), SGW_BLOCK, 0, st>>>(nG, P, gptr, gtorn, gw, g2c, ut, ldt, uc, ldc, z, ldz);
}

// ---------------------------------------------------------------------------
// K3c: Chebyshev polynomial preconditioner, the alternative to the exact
// mean-matrix solve of K3.  Per block b it returns z = p(D^{-1} A0) D^{-1} r,
// the result of `deg` steps of the Chebyshev iteration for A0 z = r with
// Jacobi scaling D = diag(A0) on the block's spectral interval [lo, hi]
// (Saad, Iterative Methods for Sparse Linear Systems, 2nd ed., Alg. 12.1),
// started from z = 0.  A0 is the mean matrix (coefficient slot k = 0).
// The result is SPD in r whenever the scaled spectrum lies in (0, lo + hi).
// One workgroup per (block, tile of Q modes): the block's rows stay in the
// workgroup for all steps, the search direction goes through LDS, the rest
// lives in registers (RPT rows per thread).  Also writes the partial sums
// part[b*P + j] = r_j'z_j over the block (and part2 = r_j'r_j if given), in a
// fixed order.
// ---------------------------------------------------------------------------
#define CHEB_TPB 1024
#define CHEB_MAX_DEG 64
#define CHEB_COEF_BYTES (2 * CHEB_MAX_DEG * 8)

// Q consecutive values of one row in an LDS direction buffer, read in the
// widest naturally aligned pieces (the row's byte offset is a multiple of
// Q * sizeof(T)).
template <typename T, int Q>
__device__ __forceinline__ void lds_read_row(const unsigned char* p, T (&v)[Q]) {
  constexpr int bytes = Q * (int)sizeof(T);
  constexpr int piece = bytes % 16 == 0 ? 16 : (bytes % 8 == 0 ? 8 : 4);
  constexpr int per = piece / (int)sizeof(T) > 0 ? piece / (int)sizeof(T) : 1;
  if constexpr (piece == 16 && sizeof(T) == 4) {
#pragma unroll
    for (int c = 0; c < Q / 4; ++c) {
      const float4 w = *reinterpret_cast<const float4*>(p + 16 * c);
      v[4 * c] = w.x; v[4 * c + 1] = w.y; v[4 * c + 2] = w.z; v[4 * c + 3] = w.w;
    }
  } else if constexpr (piece >= 8 && sizeof(T) == 4) {
#pragma unroll
    for (int c = 0; c < Q / 2; ++c) {
      const float2 w = *reinterpret_cast<const float2*>(p + 8 * c);
      v[2 * c] = w.x; v[2 * c + 1] = w.y;
    }
  } else if constexpr (piece == 16 && sizeof(T) == 8) {
#pragma unroll
    for (int c = 0; c < Q / 2; ++c) {
      const double2 w = *reinterpret_cast<const double2*>(p + 16 * c);
      v[2 * c] = w.x; v[2 * c + 1] = w.y;
    }
  } else {
    (void)per;
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = *reinterpret_cast<const T*>(p + q * sizeof(T));
  }
}

// 8 consecutive values from global memory (32-byte aligned for float,
// 64-byte for double) in 16-byte loads
template <typename T>
__device__ __forceinline__ void load_row8(const T* p, T (&v)[8]) {
  if constexpr (sizeof(T) == 4) {
    const float4 a = reinterpret_cast<const float4*>(p)[0], b = reinterpret_cast<const float4*>(p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double2 a = reinterpret_cast<const double2*>(p)[c];
      v[2 * c] = a.x;
      v[2 * c + 1] = a.y;
    }
  }
}

template <typename T, int Q>
__device__ __forceinline__ void lds_write_row(unsigned char* p, const T (&v)[Q]) {
  constexpr int bytes = Q * (int)sizeof(T);
  if constexpr (bytes % 16 == 0 && sizeof(T) == 4) {
#pragma unroll
    for (int c = 0; c < Q / 4; ++c)
      *reinterpret_cast<float4*>(p + 16 * c) =
          make_float4(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]);
  } else if constexpr (bytes % 8 == 0 && sizeof(T) == 4) {
#pragma unroll
    for (int c = 0; c < Q / 2; ++c)
      *reinterpret_cast<float2*>(p + 8 * c) = make_float2(v[2 * c], v[2 * c + 1]);
  } else if constexpr (bytes % 16 == 0 && sizeof(T) == 8) {
#pragma unroll
    for (int c = 0; c < Q / 2; ++c)
      *reinterpret_cast<double2*>(p + 16 * c) = make_double2(v[2 * c], v[2 * c + 1]);
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q) *reinterpret_cast<T*>(p + q * sizeof(T)) = v[q];
  }
}

template <typename T, int Q, int RPT, int TPB>
__global__ __launch_bounds__(TPB) void k_cheb(
    const T* __restrict__ cval, const int* __restrict__ row_off, const int* __restrict__ order,
    const int* __restrict__ crow, const unsigned short* __restrict__ cnb,
    const T* __restrict__ coef, int P, int deg,
    const T* __restrict__ r, int ldr, T* __restrict__ z, int ldz, double* __restrict__ part,
    double* __restrict__ part2, double* sc, int par, double tol2, const double* rrpart,
    int* flags, unsigned long long* acct) {
  // all LDS is dynamic (so the launch may use up to the whole 160 KiB):
  // two buffers of the search direction, each [RPT * TPB][Q] (the Q
  // modes of a row side by side, at a fixed stride, so every LDS offset but
  // the neighbour's row is a constant), the step coefficients, the
  // reduction slots
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr size_t kBuf = sizeof(T) * (size_t)RPT * TPB * Q;
  unsigned char* dir = smem_raw;
  T* cs = reinterpret_cast<T*>(smem_raw + 2 * kBuf);
  double(*red)[TPB / 64][Q] =
      reinterpret_cast<double(*)[TPB / 64][Q]>(smem_raw + 2 * kBuf + CHEB_COEF_BYTES);
  const int b = order ? order[blockIdx.x] : blockIdx.x, j0 = blockIdx.y * Q;
  if (sc) {  // stopping test of PCG iteration par, fused (see k_pcg_test)
    const double rr = sum_modes(rrpart, b, P);
    const bool act = sc[(size_t)b * 8 + 2 + par] != 0.0 && rr > tol2 * sc[(size_t)b * 8 + 4];
    if (blockIdx.y == 0 && threadIdx.x == 0) {
      sc[(size_t)b * 8 + 3 - par] = act ? 1.0 : 0.0;
      if (act) atomicAdd(&flags[0], 1);
      if (!isfinite(rr)) atomicOr(&flags[2], 1);
    }
    if (!act) return;  // converged block: its z and r'z are not used again
  }
  const int r0 = row_off[b], n = row_off[b + 1] - r0;
  if (acct && threadIdx.x == 0) {  // algorithmic bytes of this (active) workgroup
    const int nq = min(Q, P - j0);
    atomicAdd(acct, (unsigned long long)(2 * sizeof(T) * nq * n +
                                         (blockIdx.y == 0 ? 7 * (sizeof(T) + 4) * n : 0)));
  }
  // the block's step coefficients, staged in LDS (read after the first
  // barrier)
  for (int e = threadIdx.x; e < 2 * deg; e += TPB) cs[e] = coef[(size_t)b * 2 * deg + e];
  // thread i owns the row at natural (lexicographic mesh) position i of the
  // block, crow[r0 + i]; the LDS copy of the direction is in natural order,
  // so the neighbour reads and the writes of a wave are nearly contiguous
  // (few bank conflicts; measured: rows in system order with scattered LDS
  // positions take twice as long per step); cnb gives the neighbours'
  // natural positions (slot 0 is the row itself, whose value the thread
  // holds)
  unsigned lo[RPT][7];
  int row[RPT];
  T av[RPT][7], dinv[RPT];
  // the right-hand side stays in registers for the final r'z when small
  // (else it is read again)
  constexpr bool kKeepR = RPT * Q * sizeof(T) <= 24;
  T rin[kKeepR ? RPT : 1][kKeepR ? Q : 1];
  T res[RPT][Q], zz[RPT][Q], dd[RPT][Q];
  const T inv_theta = coef[(size_t)b * 2 * deg];
  // the neighbour positions and the mean-matrix row of natural position i
  // are [8]-records (16-byte loads, independent of crow)
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    const int i = threadIdx.x + t * TPB;
    const bool live = i < n;
    row[t] = live ? crow[r0 + i] : r0;
    uint4 nb4 = make_uint4(0u, 0u, 0u, 0u);
    T a8[8];
    if (live) {
      nb4 = *reinterpret_cast<const uint4*>(cnb + (size_t)(r0 + i) * 8);
      load_row8(cval + (size_t)(r0 + i) * 8, a8);
    } else {
#pragma unroll
      for (int sl = 0; sl < 8; ++sl) a8[sl] = T(0);
    }
    const unsigned nbw[4] = {nb4.x, nb4.y, nb4.z, nb4.w};
#pragma unroll
    for (int sl = 0; sl < 7; ++sl) {
      lo[t][sl] = ((nbw[sl >> 1] >> (16 * (sl & 1))) & 0xffffu) * (unsigned)(Q * sizeof(T));
      av[t][sl] = a8[sl];
    }
    dinv[t] = live ? T(1) / av[t][0] : T(0);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int j = j0 + q;
      const T v = (live && j < P) ? r[(size_t)j * ldr + row[t]] : T(0);
      if constexpr (kKeepR) rin[t][q] = v;
      res[t][q] = v;
      zz[t][q] = T(0);
      dd[t][q] = dinv[t] * v * inv_theta;
    }
  }
  // one Chebyshev step; step k writes direction buffer k & 1 (compile-time
  // offset): the buffer written two steps earlier is free because every
  // thread has passed the barrier of step k-1, after its reads of step k-2
  auto step = [&](auto bufc, int k) -> bool {
    constexpr size_t boff = decltype(bufc)::value * kBuf;
#pragma unroll
    for (int t = 0; t < RPT; ++t)
#pragma unroll
      for (int q = 0; q < Q; ++q) zz[t][q] += dd[t][q];
    if (k + 1 == deg) return true;
    unsigned char* Dk = dir + boff;
#pragma unroll
    for (int t = 0; t < RPT; ++t) {
      const int i = threadIdx.x + t * TPB;
      if (i < n) lds_write_row<T, Q>(Dk + (size_t)i * Q * sizeof(T), dd[t]);
    }
    __syncthreads();
    const T c1 = cs[2 * (k + 1)], c2 = cs[2 * (k + 1) + 1];
#pragma unroll
    for (int t = 0; t < RPT; ++t) {
      const int i = threadIdx.x + t * TPB;
      if (i >= n) continue;
      T ad[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) ad[q] = av[t][0] * dd[t][q];
#pragma unroll
      for (int sl = 1; sl < 7; ++sl) {
        T nv[Q];
        lds_read_row<T, Q>(Dk + lo[t][sl], nv);
#pragma unroll
        for (int q = 0; q < Q; ++q) ad[q] = fmadd(av[t][sl], nv[q], ad[q]);
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        res[t][q] -= ad[q];
        dd[t][q] = fmadd(c1, dd[t][q], c2 * dinv[t] * res[t][q]);
      }
    }
    return false;
  };
  for (int k = 0;; k += 2) {
    if (step(std::integral_constant<int, 0>{}, k)) break;
    if (step(std::integral_constant<int, 1>{}, k + 1)) break;
  }
  // store z; partial sums of r'z and r'r
  double srz[Q], srr[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) srz[q] = srr[q] = 0.0;
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    const int i = threadIdx.x + t * TPB;
    if (i >= n) continue;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int j = j0 + q;
      if (j >= P) continue;
      z[(size_t)j * ldz + row[t]] = zz[t][q];
      double rv;
      if constexpr (kKeepR) rv = (double)rin[t][q];
      else rv = (double)r[(size_t)j * ldr + row[t]];
      srz[q] += rv * (double)zz[t][q];
      srr[q] += rv * rv;
    }
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const double a = wave_sum(srz[q]);
    const double bq = part2 ? wave_sum(srr[q]) : 0.0;
    if (lane == 0) {
      red[0][w][q] = a;
      red[1][w][q] = bq;
    }
  }
  __syncthreads();
  if (threadIdx.x < Q && j0 + (int)threadIdx.x < P) {
    const int q = threadIdx.x;
    double a = 0.0, bq = 0.0;
    for (int v = 0; v < TPB / 64; ++v) {
      a += red[0][v][q];
      bq += red[1][v][q];
    }
    part[(size_t)b * P + j0 + q] = a;
    if (part2) part2[(size_t)b * P + j0 + q] = bq;
  }
}

void cheb_coefficients(double lo, double hi, int deg, double* out) {
  const double theta = 0.5 * (hi + lo);
  const double delta = std::max(0.5 * (hi - lo), 1e-3 * theta);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  out[0] = 1.0 / theta;
  out[1] = 0.0;
  for (int k = 1; k < deg; ++k) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    out[2 * k] = rn * rho;
    out[2 * k + 1] = 2.0 * rn / delta;
    rho = rn;
  }
}

// Launch shapes: shape 0, 1, 2 = workgroups of 1024, 512, 256 threads; each
// thread owns RPT = 1, 2 or 4 rows of the block (the smallest that covers
// the largest block); 0 if the shape cannot cover max_rows.
static int cheb_tpb(int shape) { return CHEB_TPB >> shape; }
static int cheb_rpt(int max_rows, int shape) {
  const int tpb = cheb_tpb(shape);
  return max_rows <= tpb ? 1 : (max_rows <= 2 * tpb ? 2 : (max_rows <= 4 * tpb ? 4 : 0));
}

template <typename T>
size_t cheb_lds_bytes(int max_rows, int Q, int shape) {
  const int tpb = cheb_tpb(shape);
  return sizeof(double) * 2 * (tpb / 64) * Q + CHEB_COEF_BYTES +
         2 * (size_t)cheb_rpt(max_rows, shape) * tpb * Q * sizeof(T);
}

struct ChebTest {  // optional fused stopping test (sc == nullptr: none), block order,
  const int* order;  // byte counter of timed launches (may be null)
  unsigned long long* acct;
  double* sc;
  int par;
  double tol2;
  const double* rrpart;
  int* flags;
  hipEvent_t ev0, ev1;  // timing events recorded by the launch itself (may be null)
};

struct ChebArgs {
  const int* row_off;
  const int* crow;
  const unsigned short* cnb;
  const void* coef;
  int nb, P, deg, max_rows, shape;
  const void* r;
  int ldr;
  void* z;
  int ldz;
  double *part, *part2;
};

template <typename T, int Q, int RPT, int TPB>
static void launch_cheb(const T* cval, const ChebArgs& a, const ChebTest& t, hipStream_t st) {
  dim3 grid(a.nb, ceil_div(a.P, Q));
  const unsigned lds = (unsigned)cheb_lds_bytes<T>(a.max_rows, Q, a.shape);
  if (t.ev0) {  // the dispatch records the events: kernel start and end
    hipExtLaunchKernelGGL(k_cheb<T, Q, RPT, TPB>, grid, dim3(TPB), lds, st, t.ev0, t.ev1, 0u,
                          cval, a.row_off, t.order, a.crow, a.cnb,
                          static_cast<const T*>(a.coef), a.P, a.deg,
                          static_cast<const T*>(a.r), a.ldr, static_cast<T*>(a.z), a.ldz,
                          a.part, a.part2, t.sc, t.par, t.tol2, t.rrpart, t.flags, t.acct);
    return;
  }
  k_cheb<T, Q, RPT, TPB><<<grid, TPB, lds, st>>>(
      cval, a.row_off, t.order, a.crow, a.cnb, static_cast<const T*>(a.coef), a.P, a.deg,
      static_cast<const T*>(a.r), a.ldr, static_cast<T*>(a.z), a.ldz, a.part, a.part2, t.sc,
      t.par, t.tol2, t.rrpart, t.flags, t.acct);
}

template <typename T, int RPT, int TPB>
static void cheb_q(int Q, const T* cval, const ChebArgs& a, const ChebTest& t,
                   hipStream_t st) {
  switch (Q) {
#define SGW_CHEB_CASE(q)                            \
  case q:                                          \
    launch_cheb<T, q, RPT, TPB>(cval, a, t, st);   \
    break;
    SGW_CHEB_CASE(1)
    SGW_CHEB_CASE(2)
    SGW_CHEB_CASE(3)
    SGW_CHEB_CASE(4)
    SGW_CHEB_CASE(5)
    SGW_CHEB_CASE(6)
    SGW_CHEB_CASE(7)
    default:
    SGW_CHEB_CASE(8)
#undef SGW_CHEB_CASE
  }
}

// The kernels have no static LDS, so the whole 160 KiB may be dynamic; the
// attribute is set once for every instantiation before the first launch.
template <typename T, int RPT, int TPB>
static bool cheb_attr_rpt() {
  bool ok = true;
#define SGW_CHEB_ATTR(q)                                                                \
  ok = ok && hipFuncSetAttribute((const void*)k_cheb<T, q, RPT, TPB>,                    \
                                 hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) == \
                 hipSuccess;
  SGW_CHEB_ATTR(1)
  SGW_CHEB_ATTR(2)
  SGW_CHEB_ATTR(3)
  SGW_CHEB_ATTR(4)
  SGW_CHEB_ATTR(5)
  SGW_CHEB_ATTR(6)
  SGW_CHEB_ATTR(7)
  SGW_CHEB_ATTR(8)
#undef SGW_CHEB_ATTR
  return ok;
}
template <typename T, int TPB>
static bool cheb_attr_tpb() {
  return cheb_attr_rpt<T, 1, TPB>() && cheb_attr_rpt<T, 2, TPB>() && cheb_attr_rpt<T, 4, TPB>();
}
int cheb_prepare() {
  bool ok = cheb_attr_tpb<double, CHEB_TPB>() && cheb_attr_tpb<double, CHEB_TPB / 2>() &&
            cheb_attr_tpb<double, CHEB_TPB / 4>() && cheb_attr_tpb<float, CHEB_TPB>() &&
            cheb_attr_tpb<float, CHEB_TPB / 2>() && cheb_attr_tpb<float, CHEB_TPB / 4>();
  return ok ? 0 : -1;
}

// Largest mode tile that keeps the per-thread arrays (3 x RPT x Q values
// plus the matrix rows) in registers: larger tiles spill to scratch memory
// (measured: up to 400 MB of scratch traffic per launch); 0 if the shape
// cannot cover max_rows.
template <typename T>
int cheb_max_q(int max_rows, int shape) {
  if (shape < 0 || shape > 2) return 0;
  const int rpt = cheb_rpt(max_rows, shape);
  if (rpt == 0) return 0;
  if (sizeof(T) == 8) return rpt <= 1 ? 6 : (rpt <= 2 ? 2 : 1);
  return rpt <= 1 ? 8 : (rpt <= 2 ? 4 : 2);
}

template <typename T>
int cheb_apply(const T* cval, const int* row_off, const int* order, const int* crow,
               const unsigned short* cnb, const T* coef, int nb, int P, int deg,
               int Q, int shape, int max_rows, const T* r, int ldr, T* z, int ldz,
               double* part, double* part2, double* sc, int par, double tol2,
               const double* rrpart, int* flags, unsigned long long* acct, hipStream_t st,
               hipEvent_t ev0, hipEvent_t ev1) {
  if (Q < 1 || Q > cheb_max_q<T>(max_rows, shape) || deg < 1 || deg > CHEB_MAX_DEG ||
      max_rows < 1 || cheb_lds_bytes<T>(max_rows, Q, shape) > 150 * 1024 ||
      (sc && (!rrpart || !flags)) || !crow || !cnb || !coef || !cval)
    return -1;
  const ChebTest t{order, acct, sc, par, tol2, rrpart, flags, ev1 ? ev0 : nullptr, ev1};
  const ChebArgs a{row_off, crow, cnb, coef, nb, P, deg, max_rows, shape, r, ldr, z, ldz,
                   part, part2};
  const int rpt = cheb_rpt(max_rows, shape);
#define SGW_CHEB_SHAPE(tpb)                                \
  if (rpt == 1) cheb_q<T, 1, tpb>(Q, cval, a, t, st);         \
  else if (rpt == 2) cheb_q<T, 2, tpb>(Q, cval, a, t, st);    \
  else cheb_q<T, 4, tpb>(Q, cval, a, t, st);
  if (shape == 0) {
    SGW_CHEB_SHAPE(CHEB_TPB)
  } else if (shape == 1) {
    SGW_CHEB_SHAPE(CHEB_TPB / 2)
  } else {
    SGW_CHEB_SHAPE(CHEB_TPB / 4)
  }
#undef SGW_CHEB_SHAPE
  return 0;
}

// ---------------------------------------------------------------------------
// K5: coarse grid (Eq. Fcc_2, NNCP2).  d_c = sum_s B_c^T (D_s r_c - K~^s_{c,(ir)} y^s)
// with y^s the Neumann solution; u_c = F_cc^{-1} d_c with the FP64 inverse;
// the lift adds the coarse basis Phi_s u_c^s on the remaining rows.
// ---------------------------------------------------------------------------
// d_c[m][ci]: one wave per coarse unknown (mode m, corner ci); the lanes
// share the Galerkin entries of output mode m.
template <typename T>
__global__ __launch_bounds__(SGW_BLOCK) void k_coarse_rhs(DCoarse c, const T* r, int ldr,
                                                         const T* yt, int ldt, double* dc) {
  const long long t = (long long)blockIdx.x * (SGW_BLOCK / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= (long long)c.nC * c.P) return;
  const int m = (int)(t / c.nC), ci = (int)(t % c.nC);
  const int g0 = c.gi_ptr[m], g1 = c.gi_ptr[m + 1];
  double s = 0.0;
  for (int q = c.c_ptr[ci]; q < c.c_ptr[ci + 1]; ++q) {
    const int lc = c.c_lc[q];
    if (lane == 0) s += c.sc_w[lc] * (double)r[(size_t)m * ldr + c.sc_gidx[lc]];
    for (int e = c.cc_ptr[lc]; e < c.cc_ptr[lc + 1]; ++e) {
      const int row = c.cc_torn[e];
      const double* kv = c.cc_val + (size_t)e * c.nk;
      for (int g = g0 + lane; g < g1; g += 64)
        s -= c.gi_v[g] * kv[c.gi_k[g]] * (double)yt[(size_t)c.gi_j[g] * ldt + row];
    }
  }
  s = wave_sum(s);
  if (lane == 0) dc[(size_t)m * c.nC + ci] = s;
}
template <typename T>
void coarse_rhs(const DCoarse& c, const T* r, int ldr, const T* yt, int ldt, double* dc,
                hipStream_t st) {
  long long N = (long long)c.nC * c.P;
  const int wpb = SGW_BLOCK / 64;
  if (N > 0)
    k_coarse_rhs<T><<<(int)((N + wpb - 1) / wpb), SGW_BLOCK, 0, st>>>(c, r, ldr, yt, ldt, dc);
}

// u_c = F_cc^{-1} d_c with the block-bidiagonal factor F_cc = L L^T of the
// corner rows (coarse.h): forward y_i = L_ii^{-1} (d_i - B_i y_{i-1}),
// backward x_i = L_ii^{-T} (y_i - B_{i+1}^T x_{i+1}).  Every step is a dense
// product with a stored block (the inverse diagonal blocks and their
// transposes, the sub-diagonal blocks and their transposes, all row-major):
// one wave per output row, the row read contiguously by the lanes.
// out[r] = (a ? a[r] : 0) + sign * sum_c M[r][c] v[c], c over the whole row
// (tri 0), c <= r (tri 1, lower) or c >= r (tri 2, upper).
template <typename TM>
__global__ __launch_bounds__(SGW_BLOCK) void k_coarse_gemv(int nr, int nc, const TM* M, int ld,
                                                          const double* v, const double* a,
                                                          double* out, double sign, int tri) {
  const int row = blockIdx.x * (SGW_BLOCK / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= nr) return;
  const TM* mr = M + (size_t)row * ld;
  const int c0 = tri == 2 ? row : 0, c1 = tri == 1 ? row + 1 : nc;
  // four independent partial sums: four row loads in flight per lane
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int col = c0 + lane;
  for (; col + 192 < c1; col += 256) {
    s0 += (double)mr[col] * v[col];
    s1 += (double)mr[col + 64] * v[col + 64];
    s2 += (double)mr[col + 128] * v[col + 128];
    s3 += (double)mr[col + 192] * v[col + 192];
  }
  for (; col < c1; col += 64) s0 += (double)mr[col] * v[col];
  const double s = wave_sum((s0 + s1) + (s2 + s3));
  if (lane == 0) out[row] = (a ? a[row] : 0.0) + sign * s;
}
__global__ void k_coarse_perm(int n, const int* perm, const double* src, double* dst, int gather) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= n) return;
  if (gather) dst[w] = src[perm[w]];
  else dst[perm[w]] = src[w];
}
template <typename TM>
static void coarse_sweeps(const DCoarseFactor& f, const std::vector<const TM*>& linv,
                          const std::vector<const TM*>& linvT, const std::vector<const TM*>& b,
                          const std::vector<const TM*>& bT, const double* dc, double* uc,
                          hipStream_t st) {
  const int wpb = SGW_BLOCK / 64;
  auto gemv = [&](int nr, int nc, const TM* M, const double* v, const double* a, double* out,
                  double sign, int tri) {
    k_coarse_gemv<TM><<<(nr + wpb - 1) / wpb, SGW_BLOCK, 0, st>>>(nr, nc, M, nc, v, a, out, sign,
                                                                  tri);
  };
  const std::vector<int>& o = f.off;
  k_coarse_perm<<<(f.n + 255) / 256, 256, 0, st>>>(f.n, f.perm, dc, f.wd, 1);
  for (int i = 0; i < f.R; ++i) {
    const int m = o[i + 1] - o[i];
    const double* t = f.wd + o[i];
    if (i > 0) {
      gemv(m, o[i] - o[i - 1], b[i - 1], f.wy + o[i - 1], f.wd + o[i], f.wt + o[i], -1.0, 0);
      t = f.wt + o[i];
    }
    gemv(m, m, linv[i], t, nullptr, f.wy + o[i], 1.0, 1);
  }
  for (int i = f.R - 1; i >= 0; --i) {
    const int m = o[i + 1] - o[i];
    const double* t = f.wy + o[i];
    if (i + 1 < f.R) {
      gemv(m, o[i + 2] - o[i + 1], bT[i], f.wx + o[i + 1], f.wy + o[i], f.wt + o[i], -1.0, 0);
      t = f.wt + o[i];
    }
    gemv(m, m, linvT[i], t, nullptr, f.wx + o[i], 1.0, 2);
  }
  k_coarse_perm<<<(f.n + 255) / 256, 256, 0, st>>>(f.n, f.perm, f.wx, uc, 0);
}
void coarse_solve(const DCoarseFactor& f, const double* dc, double* uc, bool single,
                  hipStream_t st) {
  if (f.n <= 0) return;
  if (single && !f.linvf.empty())
    coarse_sweeps<float>(f, f.linvf, f.linvTf, f.bf, f.bTf, dc, uc, st);
  else
    coarse_sweeps<double>(f, f.linv, f.linvT, f.b, f.bT, dc, uc, st);
}

// ut[j][rem] += sum_{m, lc} Phi_s[(m, lc)][(j, tr)] uc[m][coarse(lc)]: the
// subdomain's coarse values go to LDS, each thread owns one output and
// streams its column of Phi_s (contiguous across the threads).  The FP32
// path reads an FP16 copy of Phi (half the bytes of this bandwidth-bound
// product; the lift belongs to the preconditioner, whose Neumann solves in
// that path stop at a relative residual of 1e-2, far above FP16 rounding).
template <typename T>
__global__ __launch_bounds__(SGW_BLOCK) void k_coarse_lift(DCoarse c, const double* uc, T* ut,
                                                          int ldt) {
  __shared__ double ucl[SGW_MAX_COARSE_LOCAL];
  const int s = blockIdx.x;
  const int nrem = c.rem_off[s + 1] - c.rem_off[s];
  const int lc0 = c.sc_ptr[s], ncs = c.sc_ptr[s + 1] - lc0;
  if (ncs == 0) return;
  const int nq = c.P * ncs;
  for (int q = threadIdx.x; q < nq; q += SGW_BLOCK)
    ucl[q] = uc[(size_t)(q / ncs) * c.nC + c.sc_coarse[lc0 + q % ncs]];
  __syncthreads();
  const long long nout = (long long)c.P * nrem;
  if constexpr (sizeof(T) == 4) {
    // four consecutive outputs per thread: one 8-byte load of four FP16
    // values per coarse unknown (rows padded to a multiple of 4)
    const long long npad = (nout + 3) / 4 * 4;
    const long long o = 4 * ((long long)blockIdx.y * SGW_BLOCK + threadIdx.x);
    if (o >= nout) return;
    const uint2* ph = reinterpret_cast<const uint2*>(c.phih + c.phih_off[s] + o);
    const long long stride = npad / 4;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll 4
    for (int q = 0; q < nq; ++q) {
      const uint2 v = ph[(size_t)q * stride];
      const double u = ucl[q];
      a0 += (double)(float)__builtin_bit_cast(_Float16, (unsigned short)(v.x & 0xffffu)) * u;
      a1 += (double)(float)__builtin_bit_cast(_Float16, (unsigned short)(v.x >> 16)) * u;
      a2 += (double)(float)__builtin_bit_cast(_Float16, (unsigned short)(v.y & 0xffffu)) * u;
      a3 += (double)(float)__builtin_bit_cast(_Float16, (unsigned short)(v.y >> 16)) * u;
    }
    const double acc[4] = {a0, a1, a2, a3};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (o + e >= nout) break;
      const int j = (int)((o + e) / nrem), tr = (int)((o + e) % nrem);
      T* dst = ut + (size_t)j * ldt + c.rem_list[c.rem_off[s] + tr];
      *dst = (T)((double)*dst + acc[e]);
    }
  } else {
    const long long o = (long long)blockIdx.y * SGW_BLOCK + threadIdx.x;
    if (o >= nout) return;
    double acc = 0.0;
    const double* ph = c.phi + c.phi_off[s] + o;
#pragma unroll 8
    for (int q = 0; q < nq; ++q) acc += ph[(size_t)q * nout] * ucl[q];
    const int j = (int)(o / nrem), tr = (int)(o % nrem);
    T* dst = ut + (size_t)j * ldt + c.rem_list[c.rem_off[s] + tr];
    *dst = (T)((double)*dst + acc);
  }
}
// per subdomain: rows of nout values of phi -> rows of npad FP16 values (zeros after nout)
__global__ void k_basis_to_half(DCoarse c, const int* nq_s, const long long* nout_s) {
  const int s = blockIdx.y;
  const long long nout = nout_s[s], npad = (nout + 3) / 4 * 4;
  const long long tot = (long long)nq_s[s] * npad;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
       i += (long long)gridDim.x * blockDim.x) {
    const long long q = i / npad, o = i - q * npad;
    const float v = o < nout ? (float)c.phi[c.phi_off[s] + q * nout + o] : 0.0f;
    const_cast<unsigned short*>(c.phih)[c.phih_off[s] + i] = __builtin_bit_cast(unsigned short, (_Float16)v);
  }
}
void coarse_basis_to_half(const DCoarse& c, int nsub, const int* nq, const long long* nout,
                          hipStream_t st) {
  if (c.nC == 0 || nsub <= 0) return;
  k_basis_to_half<<<dim3(256, nsub), 256, 0, st>>>(c, nq, nout);
}
template <typename T>
void coarse_lift(const DCoarse& c, int nsub, const double* uc, T* ut, int ldt, hipStream_t st) {
  if (c.nC == 0) return;
  const long long per = sizeof(T) == 4 ? 4 : 1;  // outputs per thread
  const int gy = (int)((c.P * (long long)c.max_rem + per * SGW_BLOCK - 1) / (per * SGW_BLOCK));
  k_coarse_lift<T><<<dim3(nsub, std::max(gy, 1)), SGW_BLOCK, 0, st>>>(c, uc, ut, ldt);
}

// explicit instantiations
template size_t tri_lds_bytes<double>(const DFactor&, int);
template size_t cheb_lds_bytes<double>(int, int, int);
template int cheb_max_q<double>(int, int);
template int cheb_max_q<float>(int, int);
template size_t cheb_lds_bytes<float>(int, int, int);
template int cheb_apply<double>(const double*, const int*, const int*, const int*,
                                const unsigned short*, const double*, int, int, int,
                                int, int, int, const double*, int, double*, int, double*, double*,
                                double*, int, double, const double*, int*, unsigned long long*,
                                hipStream_t, hipEvent_t, hipEvent_t);
template int cheb_apply<float>(const float*, const int*, const int*, const int*,
                               const unsigned short*, const float*, int, int, int,
                               int, int, int, const float*, int, float*, int, double*, double*,
                               double*, int, double, const double*, int*, unsigned long long*,
                               hipStream_t, hipEvent_t, hipEvent_t);
template size_t tri_lds_bytes<float>(const DFactor&, int);
#define SGW_INST(T)                                                                          \
  template void sg_apply<T>(const DEll<T>&, const GTab&, const DHalo*, int, int, const T*,    \
                            int, T*, int, T, T, int, long long, long long, hipStream_t);    \
  template void mass_apply<T>(const DEll<T>&, int, int, int, const T*, int, T*, int, T, T,   \
                              hipStream_t);                                                  \
  template void tri_solve<T>(const DFactor&, int, const T*, int, T*, int, int, long long,    \
                             long long, hipStream_t);                                        \
  template void seg_dot<T>(int, const int*, int, const T*, int, const T*, int, double*,     \
                           const T*, int, const T*, int, double*, hipStream_t);             \
  template void pcg_xr<T>(int, const int*, int, int, double*, T*, int, const T*, int, \
                          T*, int, const T*, int, const double*, double*, int*,            \
                          hipStream_t, const int*, int);                                     \
  template bool sg_apply_pcg_fits<T>(const GTab&, const DHalo&);                             \
  template bool sg_apply_pcg<T>(const DEll<T>&, const GTab&, const DHalo&, int, const T*,    \
                                const T*, T*, int, T*, const double*, double*, int, double*, \
                                unsigned long long*, unsigned, hipStream_t);                 \
  template void pcg_p<T>(int, const int*, int, int, double*, const double*, const T*, int,  \
                         T*, int, hipStream_t);                                              \
  template void fill2d<T>(int, int, T*, int, T, hipStream_t);                               \
  template void axpby2d<T>(int, int, double, const T*, int, double, const T*, int, T*, int, \
                           hipStream_t);                                                     \
  template void axpby2d_dev<T>(int, int, double, int, const T*, int, double, int, const T*,  \
                               int, T*, int, const double*, hipStream_t);                    \
  template void scatter_to_torn<T>(int, int, const int*, const double*, const T*, int, T*,  \
                                   int, hipStream_t);                                        \
  template void gather_from_torn<T>(int, int, const int*, const int*, const double*,        \
                                    const int*, const T*, int, const double*, int, T*, int,  \
                                    hipStream_t);                                            \
  template void coarse_rhs<T>(const DCoarse&, const T*, int, const T*, int, double*,        \
                              hipStream_t);                                                  \
  template void coarse_lift<T>(const DCoarse&, int, const double*, T*, int, hipStream_t);
SGW_INST(double)
SGW_INST(float)
template void copy2d<double, double>(int, int, const double*, int, double*, int, double, hipStream_t);
template void copy2d<float, double>(int, int, const double*, int, float*, int, double, hipStream_t);
template void copy2d<double, float>(int, int, const float*, int, double*, int, double, hipStream_t);
template void copy2d<float, float>(int, int, const float*, int, float*, int, double, hipStream_t);

}  // namespace k
}  // namespace sgw
