// Banded LDL^T factorisation and solve by one workgroup.
//
// B holds the lower band of a symmetric matrix of n rows and bandwidth b:
// row l, column l-t (0 <= t <= b) at B[l*(b+1) + b - t].  X holds nck
// right-hand sides, row-major [n][nck].  The factorisation is right-looking:
// at step k, d_k = B(k,k) and every entry (k+t, k+s), 1 <= s <= t <= b, loses
// B(k+t,k) B(k+s,k) / d_k; the column below d_k is left unscaled (it holds
// L(.,k) d_k), so the forward sweep uses B(k+t,k)/d_k and the backward sweep
// x_k = (z_k - sum_t B(k+t,k) x_{k+t}) / d_k.  One barrier per step.
// Returns true if a pivot was not positive (the matrix is then not SPD).
#pragma once

#include <hip/hip_runtime.h>

namespace fams {

template <class TC>
__device__ bool band_ldlt_solve(TC* B, int n, int b, TC* X, int nck) {
  const int w = b + 1;
  bool bad = false;
  for (int k = 0; k < n; ++k) {
    TC piv = B[static_cast<int64_t>(k) * w + b];
    if (!(piv > TC(0))) bad = true;
    TC rpiv = TC(1) / piv;
    int m = min(b, n - 1 - k);
    int pairs = m * m;
    int tot = pairs + m * nck;
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
      if (idx < pairs) {
        int t = idx / m + 1, s = idx % m + 1;
        if (s <= t) {
          TC lt = B[static_cast<int64_t>(k + t) * w + b - t];
          TC ls = B[static_cast<int64_t>(k + s) * w + b - s];
          B[static_cast<int64_t>(k + t) * w + b - (t - s)] -= lt * ls * rpiv;
        }
      } else {
        int u = idx - pairs;
        int t = u / nck + 1, c = u % nck;
        TC lt = B[static_cast<int64_t>(k + t) * w + b - t];
        X[static_cast<int64_t>(k + t) * nck + c] -= lt * X[static_cast<int64_t>(k) * nck + c] * rpiv;
      }
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    TC rpiv = TC(1) / B[static_cast<int64_t>(k) * w + b];
    int m = min(b, k);
    for (int idx = threadIdx.x; idx < m * nck; idx += blockDim.x) {
      int t = idx / nck + 1, c = idx % nck;
      TC xk = X[static_cast<int64_t>(k) * nck + c] * rpiv;
      X[static_cast<int64_t>(k - t) * nck + c] -= B[static_cast<int64_t>(k) * w + b - t] * xk;
    }
    __syncthreads();
  }
  for (int64_t t = threadIdx.x; t < static_cast<int64_t>(n) * nck; t += blockDim.x) {
    int k = static_cast<int>(t / nck);
    X[t] /= B[static_cast<int64_t>(k) * w + b];
  }
  __syncthreads();
  return bad;
}

}  // namespace fams
