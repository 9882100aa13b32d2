// Dense symmetric eigensolver of libdmrg (host, FP64): Householder reduction to tridiagonal form,
// then the implicit symmetric QR iteration with Wilkinson shifts (Golub and Van Loan, "Matrix
// Computations", Sections 8.3.1-8.3.3). Used for the M-state cut of Section 2.1 (eigenvectors of
// the reduced density matrices) and for Davidson's small Rayleigh-Ritz problems.
#pragma once
#include <vector>

namespace dmrg {

// Eigen-decomposition of the symmetric n x n matrix `a` (row-major; only its lower triangle is
// read). On return `evals` (n) holds the eigenvalues in ascending order and `vecs_t` (n x n,
// row-major) the matching orthonormal eigenvectors as ROWS: row k is the eigenvector of evals[k].
// `threads` > 1 spreads the eigenvector updates over that many host threads (same results for any
// count). Throws dmrg::Error(DMRG_ERR_NAN) on non-finite input or when the QR iteration does not
// converge within 30 n steps.
void sym_eigen(int n, const double* a, std::vector<double>& evals, std::vector<double>& vecs_t, int threads = 1);

}  // namespace dmrg
