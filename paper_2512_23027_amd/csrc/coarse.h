// Factor of the coarse-grid matrix F_cc of the two-level Neumann-Neumann
// preconditioner (Eq. Fcc_2), host side.
//
// The corners of a rectilinear partition sit on a grid whose rows are the
// interior cut lines y = const; a corner couples only to the corners of the
// subdomains around it, i.e. to corners of its own row and of the two
// neighbouring rows.  Ordering the coarse unknowns row by row (inside a row:
// corner by corner, the P modes of a corner contiguous) makes F_cc block
// tridiagonal with dense row blocks.  Its Cholesky factor is block
// bidiagonal, F = L L^T with
//   L_ii L_ii^T = A_ii - B_i B_i^T,   B_{i+1} = L_{i+1,i} = A_{i+1,i} L_ii^{-T}.
// The device solve needs only the inverse diagonal blocks and the
// sub-diagonal blocks: every step of its forward and backward substitution
// is then a dense matrix-vector product (no sequential triangular solve).
#pragma once
#include <string>
#include <vector>

namespace sgw {

struct CoarseBlocks {
  int R = 0;                        // corner rows
  std::vector<int> off;             // R + 1 unknown offsets of the rows
  std::vector<std::vector<double>> diag;  // A_ii, row-major m_i x m_i (full)
  std::vector<std::vector<double>> sub;   // A_{i+1,i}, m_{i+1} x m_i (entry i of R-1)
};

struct CoarseFactor {
  int R = 0;
  std::vector<int> off;
  std::vector<std::vector<double>> linv;  // L_ii^{-1}, row-major, zero above the diagonal
  std::vector<std::vector<double>> b;     // B_{i+1} = L_{i+1,i}, m_{i+1} x m_i
};

// Block-tridiagonal Cholesky of an SPD matrix given by its row blocks, with
// the inverse diagonal factor blocks.  Dense kernels run on up to `threads`
// host threads.  Returns false (message in err) on a non-positive pivot.
bool coarse_factor(const CoarseBlocks& A, CoarseFactor& F, int threads, std::string& err);

}  // namespace sgw
