// Host FP64 symmetric eigensolver (see eig.cpp).
#pragma once

namespace pts {

// d leading eigenpairs of the symmetric n x n matrix C (row-major, FP64):
// evals [d] descending, evecs [n][d] row-major (column j = j-th eigenvector,
// largest-magnitude entry positive).  nthreads <= 0: up to 16 host threads.
// Returns 0, or -1 on bad sizes.
int eig_sym_top(const double* C, int n, int d, double* evals, double* evecs, int nthreads);

}  // namespace pts
