// Launch interface of the block-Jacobi kernels (precond.hip): the Cholesky
// factor of every tile's diagonal block of D-hat + B-hat^T N^-1 B-hat and its
// application to a pixel vector.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sympix {

// For every tile J: A_J = D[dblk[J]] + C[dblk[J]] (C may be null: A_J =
// D[dblk[J]]), blocks of 64 x 64 float64 row-major at 4096 doubles per block
// index; U + 4096 J receives the upper factor (A_J = U^T U from the upper
// triangle of A_J, row-major, zeros below the diagonal) and info[J] 0, or
// j + 1 for the first pivot j that is not positive.
hipError_t launch_factor_diag(const double *D, const double *C, const int32_t *dblk, int64_t ntiles, double *U,
                              int32_t *info, hipStream_t st);

// x_J = (U_J^T U_J)^-1 r_J for every tile J (64 pixels each); x may equal r.
hipError_t launch_solve_diag(const double *U, const double *r, double *x, int64_t ntiles, hipStream_t st);

}  // namespace sympix
