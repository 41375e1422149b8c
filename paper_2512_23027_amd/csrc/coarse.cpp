// Block-tridiagonal Cholesky of the coarse-grid matrix F_cc (host, FP64).
// See coarse.h for the structure; the dense kernels below are plain
// row-major loops, split over host threads by rows (or columns) of their
// output so that every thread writes disjoint memory.
#include "coarse.h"

#include <algorithm>
#include <cmath>
#include <thread>

namespace sgw {
namespace {

template <class Fn>
void parallel_for(int n, int threads, Fn fn) {
  threads = std::max(1, std::min(threads, n));
  if (threads == 1) {
    fn(0, n);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(threads);
  for (int t = 0; t < threads; ++t) {
    const int a = (int)((long long)n * t / threads), b = (int)((long long)n * (t + 1) / threads);
    th.emplace_back([=] { fn(a, b); });
  }
  for (auto& x : th) x.join();
}

// C[m x n] = beta C + alpha A[m x k] B[n x k]^T (row-major, leading
// dimensions lda, ldb, ldc); rows of C in blocks of 4 per thread, 4 x 4
// output tiles, the k loop contiguous in A and B.
void gemm_nt(int m, int n, int k, double alpha, const double* A, int lda, const double* B,
             int ldb, double beta, double* C, int ldc, int threads) {
  const int mb = (m + 3) / 4;
  parallel_for(mb, threads, [&](int b0, int b1) {
    for (int ib = b0; ib < b1; ++ib) {
      const int i0 = 4 * ib, ni = std::min(4, m - i0);
      for (int j0 = 0; j0 < n; j0 += 4) {
        const int nj = std::min(4, n - j0);
        double s[4][4] = {};
        if (ni == 4 && nj == 4) {
          const double *a0 = A + (size_t)i0 * lda, *a1 = a0 + lda, *a2 = a1 + lda, *a3 = a2 + lda;
          const double *q0 = B + (size_t)j0 * ldb, *q1 = q0 + ldb, *q2 = q1 + ldb, *q3 = q2 + ldb;
          for (int p = 0; p < k; ++p) {
            const double x0 = a0[p], x1 = a1[p], x2 = a2[p], x3 = a3[p];
            const double y0 = q0[p], y1 = q1[p], y2 = q2[p], y3 = q3[p];
            s[0][0] += x0 * y0; s[0][1] += x0 * y1; s[0][2] += x0 * y2; s[0][3] += x0 * y3;
            s[1][0] += x1 * y0; s[1][1] += x1 * y1; s[1][2] += x1 * y2; s[1][3] += x1 * y3;
            s[2][0] += x2 * y0; s[2][1] += x2 * y1; s[2][2] += x2 * y2; s[2][3] += x2 * y3;
            s[3][0] += x3 * y0; s[3][1] += x3 * y1; s[3][2] += x3 * y2; s[3][3] += x3 * y3;
          }
        } else {
          for (int a = 0; a < ni; ++a)
            for (int b = 0; b < nj; ++b) {
              const double* x = A + (size_t)(i0 + a) * lda;
              const double* y = B + (size_t)(j0 + b) * ldb;
              double t = 0.0;
              for (int p = 0; p < k; ++p) t += x[p] * y[p];
              s[a][b] = t;
            }
        }
        for (int a = 0; a < ni; ++a)
          for (int b = 0; b < nj; ++b) {
            double& c = C[(size_t)(i0 + a) * ldc + j0 + b];
            c = (beta == 0.0 ? 0.0 : beta * c) + alpha * s[a][b];
          }
      }
    }
  });
}

// In-place lower Cholesky of the n x n row-major matrix A (the strict upper
// triangle is not referenced and is set to zero): right-looking, panels of
// NB columns, trailing update by gemm_nt on the lower block rows.
bool chol_lower(int n, double* A, int lda, int threads) {
  const int NB = 64;
  for (int j0 = 0; j0 < n; j0 += NB) {
    const int nb = std::min(NB, n - j0);
    // diagonal block (already updated by the earlier panels)
    for (int j = j0; j < j0 + nb; ++j) {
      double d = A[(size_t)j * lda + j];
      for (int p = j0; p < j; ++p) d -= A[(size_t)j * lda + p] * A[(size_t)j * lda + p];
      if (!(d > 0.0)) return false;
      d = std::sqrt(d);
      A[(size_t)j * lda + j] = d;
      for (int i = j + 1; i < j0 + nb; ++i) {
        double s = A[(size_t)i * lda + j];
        for (int p = j0; p < j; ++p) s -= A[(size_t)i * lda + p] * A[(size_t)j * lda + p];
        A[(size_t)i * lda + j] = s / d;
      }
    }
    // panel below the diagonal block: rows i solve x L_jj^T = a
    const int r0 = j0 + nb;
    parallel_for(n - r0, threads, [&](int a, int b) {
      for (int i = r0 + a; i < r0 + b; ++i) {
        double* ai = A + (size_t)i * lda;
        for (int j = j0; j < j0 + nb; ++j) {
          double s = ai[j];
          const double* lj = A + (size_t)j * lda;
          for (int p = j0; p < j; ++p) s -= ai[p] * lj[p];
          ai[j] = s / lj[j];
        }
      }
    });
    // trailing update of the lower part, block row by block row
    for (int i0 = r0; i0 < n; i0 += 256) {
      const int mi = std::min(256, n - i0);
      gemm_nt(mi, i0 + mi - r0, nb, -1.0, A + (size_t)i0 * lda + j0, lda,
              A + (size_t)r0 * lda + j0, lda, 1.0, A + (size_t)i0 * lda + r0, lda, threads);
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) A[(size_t)i * lda + j] = 0.0;
  return true;
}

// X = L^{-1} for a lower-triangular row-major L: column j of X solves
// L x = e_j by forward substitution (x_i = 0 for i < j); columns are
// independent and go to different threads.
void trtri_lower(int n, const double* L, int ldl, double* X, int ldx, int threads) {
  parallel_for(n, threads, [&](int a, int b) {
    std::vector<double> x(n);
    for (int j = a; j < b; ++j) {
      for (int i = j; i < n; ++i) {
        const double* li = L + (size_t)i * ldl;
        double s = i == j ? 1.0 : 0.0;
        for (int p = j; p < i; ++p) s -= li[p] * x[p];
        x[i] = s / li[i];
      }
      for (int i = 0; i < n; ++i) X[(size_t)i * ldx + j] = i < j ? 0.0 : x[i];
    }
  });
}

}  // namespace

bool coarse_factor(const CoarseBlocks& A, CoarseFactor& F, int threads, std::string& err) {
  F.R = A.R;
  F.off = A.off;
  F.linv.assign(A.R, {});
  F.b.assign(A.R > 0 ? A.R - 1 : 0, {});
  std::vector<double> L;
  for (int i = 0; i < A.R; ++i) {
    const int m = A.off[i + 1] - A.off[i];
    L = A.diag[i];
    if (i > 0) {  // A_ii - B_i B_i^T
      const int mp = A.off[i] - A.off[i - 1];
      const std::vector<double>& B = F.b[i - 1];
      gemm_nt(m, m, mp, -1.0, B.data(), mp, B.data(), mp, 1.0, L.data(), m, threads);
    }
    if (!chol_lower(m, L.data(), m, threads)) {
      err = "coarse matrix F_cc is not positive definite (corner row " + std::to_string(i) + ")";
      return false;
    }
    F.linv[i].assign((size_t)m * m, 0.0);
    trtri_lower(m, L.data(), m, F.linv[i].data(), m, threads);
    if (i + 1 < A.R) {  // B_{i+1} = A_{i+1,i} L_ii^{-T}
      const int mn = A.off[i + 2] - A.off[i + 1];
      F.b[i].assign((size_t)mn * m, 0.0);
      gemm_nt(mn, m, m, 1.0, A.sub[i].data(), m, F.linv[i].data(), m, 0.0, F.b[i].data(), m,
              threads);
    }
  }
  return true;
}

}  // namespace sgw
