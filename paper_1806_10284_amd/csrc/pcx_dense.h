// Small dense Hermitian linear algebra on the host (FP64, row-major).
#pragma once

#include <complex>
#include <vector>

namespace pcx {

using zc = std::complex<double>;

void hermitize(int k, std::vector<zc>& A);
// A = V diag(w) V^H, w ascending (all k); V is k x ncols, the eigenvectors of the ncols lowest
// eigenvalues (ncols < 0: all); false if the QL iteration fails to converge
bool herm_eig(int k, std::vector<zc> A, std::vector<double>& w, std::vector<zc>& V, int ncols = -1);
// G = L L^H; false if a pivot is <= rel_tol * max diag
bool cholesky(int k, const std::vector<zc>& G, std::vector<zc>& L, double rel_tol);
void solve_LH(int k, const std::vector<zc>& L, const std::vector<zc>& B, int m, std::vector<zc>& X);
void solve_L(int k, const std::vector<zc>& L, const std::vector<zc>& B, int m, std::vector<zc>& X);
// lowest `want` Ritz pairs of the pencil (GA, GB): C (k x want) with C^H GB C = I
bool rayleigh_ritz(int k, std::vector<zc> GA, std::vector<zc> GB, int want, double chol_tol,
                   std::vector<double>& theta, std::vector<zc>& C);
// C such that Y C has orthonormal columns, from G = Y^H Y
void orthonormalizer(int m, std::vector<zc> G, std::vector<zc>& C);

}  // namespace pcx
