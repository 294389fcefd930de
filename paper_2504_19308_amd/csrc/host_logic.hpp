// Host-side logic of the library with no device code: the circulant
// frequency selection, the small dense factorisations of the randomized SVD's
// host path, and the overlap test of pitched operands.  Kept free of HIP so
// that it builds with a plain C++ compiler (the host sanitizer tests do).
#ifndef AMM_HOST_LOGIC_HPP
#define AMM_HOST_LOGIC_HPP

#include <cstdint>
#include <vector>

namespace amm {

// Closed-set frequency selection (Alg. 2.3 steps 2-3 with the reading of
// amm.h): among frequency sets closed under k -> n-k with at most K members,
// the one with the largest total energy (ties: the larger set; pairs ranked by
// E[k] + E[n-k], ties to the smaller k).  Ascending order.
std::vector<int32_t> select_closed(const std::vector<double>& E, int K);
// energy kept by select_closed(E, K) for every K = 0..n
std::vector<double> retained_all(const std::vector<double>& E);

// Upper Cholesky factor in place, G = R^T R (row-major l x l; the strict
// lower part is zeroed); false if a pivot is not positive.
bool cholesky_upper(std::vector<double>& G, int l);
// inverse of an upper-triangular R (row-major l x l)
std::vector<double> inv_upper(const std::vector<double>& R, int l);
// cyclic Jacobi: symmetric G = W diag(lam) W^T (row-major, columns of W the vectors)
void jacobi_eig(std::vector<double> G, int l, std::vector<double>& lam, std::vector<double>& W);

// Whether two row panels of p floats (rows at a + i lda, i < ra, and at
// b + k ldb, k < rb) share an element (exact for equal pitches and a
// whole-float offset, else by address ranges).
bool panels_overlap(const float* a, int64_t ra, int64_t lda, const float* b, int64_t rb, int64_t ldb, int64_t p);

}  // namespace amm

#endif
