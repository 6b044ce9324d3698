// DIIS subspace solve of the amplitude iteration (P. Pulay, Chem. Phys. Lett. 73, 393 (1980)).
// Host-only C++ (no HIP): the library includes it, and so does the sanitizer build of the
// host logic that checks it on the CPU.
#ifndef PPL_DIIS_SOLVE_H
#define PPL_DIIS_SOLVE_H

#include <algorithm>
#include <cmath>
#include <vector>

namespace ppl {

// DIIS coefficients of the subspace `ids` (oldest first; slot numbers below CAP) from the
// inner products B of the error vectors: the system [B -1; -1^T 0][c; lambda] = [0; -1],
// with B divided by its largest diagonal entry, by Gaussian elimination with partial
// pivoting. Singular (false) when a pivot falls below 1e-14 or the result is not finite;
// false as well for an empty or oversized subspace or a slot outside [0, CAP).
template <int CAP>
bool diis_solve(const double (&B)[CAP][CAP], const std::vector<int>& ids, double* c) {
  const int n = (int)ids.size(), N = n + 1;
  if (n < 1 || n > CAP) return false;
  for (int i = 0; i < n; ++i)
    if (ids[i] < 0 || ids[i] >= CAP) return false;
  double scale = 0.0;
  for (int i = 0; i < n; ++i) scale = std::max(scale, std::fabs(B[ids[i]][ids[i]]));
  if (!(scale > 0.0) || !std::isfinite(scale)) return false;
  double A[CAP + 1][CAP + 2];
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) A[i][j] = B[ids[i]][ids[j]] / scale;
    A[i][n] = -1.0;
    A[n][i] = -1.0;
    A[i][N] = 0.0;
  }
  A[n][n] = 0.0;
  A[n][N] = -1.0;
  for (int col = 0; col < N; ++col) {
    int piv = col;
    for (int r = col + 1; r < N; ++r)
      if (std::fabs(A[r][col]) > std::fabs(A[piv][col])) piv = r;
    if (!(std::fabs(A[piv][col]) >= 1e-14)) return false;
    if (piv != col)
      for (int k = 0; k <= N; ++k) std::swap(A[piv][k], A[col][k]);
    for (int r = col + 1; r < N; ++r) {
      const double f = A[r][col] / A[col][col];
      for (int k = col; k <= N; ++k) A[r][k] -= f * A[col][k];
    }
  }
  double x[CAP + 1];
  for (int r = N - 1; r >= 0; --r) {
    double acc = A[r][N];
    for (int k = r + 1; k < N; ++k) acc -= A[r][k] * x[k];
    x[r] = acc / A[r][r];
  }
  for (int i = 0; i < n; ++i) {
    if (!std::isfinite(x[i])) return false;
    c[i] = x[i];
  }
  return true;
}

}  // namespace ppl

#endif
