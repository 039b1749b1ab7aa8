// Banded LDL^T factorisation and solve by one workgroup.
//
// Storage: the lower band of a symmetric matrix of n rows and bandwidth b,
// row l, column l-t (0 <= t <= b) at B[l*(b+1) + b - t].  X holds nck
// right-hand sides, row-major [n][nck].  After factorisation the diagonal
// holds D and the entries below it the unit-lower L.
//
// Three storage modes (band_mode):
//   0  the whole band in LDS: unblocked right-looking elimination in place;
//   1  band in global memory, blocked by kPanel columns, with a ring of
//      b + kPanel band rows in LDS -- each row is read once when a panel first
//      reaches it and written once when it is final;
//   2  band in global memory, blocked, trailing updates in global memory.
// Blocked steps, for the columns [k, k+nb): copy the panel (rows k..k+nb+b-1)
// to LDS, eliminate its nb columns there, write D and L back, then subtract
// the panel's rank-nb product from the trailing triangle of b rows.
// Substitution: see band_substitute.
// Functions return true if a pivot was not positive (matrix not SPD).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fams {

// Workgroup barrier that orders LDS only: waits for the wave's LDS accesses
// (lgkmcnt) but not for its global loads and stores, which may stay in
// flight across it.  For barriers that publish LDS data only.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

constexpr int kPanel = 16;   // columns per panel of the blocked factorisation
constexpr int kPanelRowsPerThread = 2;  // panels of up to 2 * 256 rows held in registers
constexpr int kSubRows = 8;  // rows per block of the substitution

__host__ __device__ inline int64_t band_panel_elems(int b) {  // P and Q of a panel
  return static_cast<int64_t>(kPanel + b) * (kPanel + 1) + static_cast<int64_t>(kPanel) * (kPanel + b);
}
__host__ __device__ inline int64_t band_ring_elems(int b) {
  return static_cast<int64_t>(kPanel + b) * (b + 1);
}
__host__ __device__ inline int64_t band_subst_elems(int b) {
  return static_cast<int64_t>(b + kSubRows) * kSubRows + kSubRows;
}

// storage mode for a band of n rows and bandwidth b with `lds` elements of
// LDS available; -1 if none fits
__host__ __device__ inline int band_mode(int n, int b, int64_t lds) {
  const int64_t sub = band_subst_elems(b);
  if (static_cast<int64_t>(n) * (b + 1) + sub <= lds) return 0;
  const int64_t pan = band_panel_elems(b);
  if (band_ring_elems(b) + pan <= lds) return 1;
  if (pan <= lds && sub <= lds) return 2;
  return -1;
}
// LDS elements that mode `mode` uses
__host__ __device__ inline int64_t band_lds_elems(int mode, int n, int b) {
  const int64_t sub = band_subst_elems(b);
  if (mode == 0) return static_cast<int64_t>(n) * (b + 1) + sub;
  const int64_t pan = band_panel_elems(b);
  if (mode == 1) return band_ring_elems(b) + pan;
  return pan > sub ? pan : sub;
}

// right-looking factorisation of B in place (B in LDS or global memory).
// Wavefronts take the rows k+t of the update, lanes the columns k+s (s <= t).
template <class TC>
__device__ bool band_factor_inplace(TC* B, int n, int b) {
  const int w = b + 1;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, nwaves = blockDim.x / 64;
  bool bad = false;
  for (int k = 0; k < n; ++k) {
    const TC piv = B[static_cast<int64_t>(k) * w + b];
    if (!(piv > TC(0))) bad = true;
    const TC rpiv = TC(1) / piv;
    const int m = min(b, n - 1 - k);
    for (int t = 1 + wave; t <= m; t += nwaves) {
      TC* row = B + static_cast<int64_t>(k + t) * w;
      const TC lt = row[b - t] * rpiv;
      for (int s = 1 + lane; s <= t; s += 64)
        row[b - (t - s)] -= lt * B[static_cast<int64_t>(k + s) * w + b - s];
    }
    lds_barrier();
  }
  return bad;
}

// turn the unscaled columns into unit-lower L: B(r, r-t) /= d_{r-t}
template <class TC>
__device__ void band_normalise(TC* B, int n, int b) {
  const int w = b + 1;
  for (int64_t e = threadIdx.x; e < static_cast<int64_t>(n) * w; e += blockDim.x) {
    const int r = static_cast<int>(e / w), t = b - static_cast<int>(e % w);
    if (t > 0 && r - t >= 0) B[e] /= B[static_cast<int64_t>(r - t) * w + b];
  }
  lds_barrier();
}

// Blocked factorisation of the band G in global memory (mode 1 / 2 above).
// LDS: the panel P [(kPanel + b) rows][kPanel + 1], its scaled transpose
// Q [kPanel][kPanel + b] (Q[c][i] = P[i][c] / d_c) and, in mode 1, the ring
// of b + kPanel band rows (row r in slot r mod (b + kPanel)).
template <class TC, bool kRing>
__device__ bool band_factor_blocked(TC* G, int n, int b, TC* lds) {
  const int w = b + 1;
  constexpr int PS = kPanel + 1;
  const int mrow = kPanel + b;
  TC* P = lds;
  TC* Q = P + static_cast<int64_t>(mrow) * PS;
  TC* ring = Q + static_cast<int64_t>(kPanel) * mrow;
  __shared__ TC colbuf[2 * kPanel];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, nwaves = blockDim.x / 64;
  auto rowp = [&](int r) -> TC* {
    if constexpr (kRing) return ring + static_cast<int64_t>(r % mrow) * w;
    else return G + static_cast<int64_t>(r) * w;
  };
  bool bad = false;
  if constexpr (kRing) {  // rows 0..b-1 enter before the first panel
    for (int64_t e = threadIdx.x; e < static_cast<int64_t>(min(n, b)) * w; e += blockDim.x)
      ring[e] = G[e];
  }
  for (int k = 0; k < n; k += kPanel) {
    const int nb = min(kPanel, n - k);
    const int np = min(n - k, nb + b);  // panel rows k .. k+np-1
    if constexpr (kRing) {  // rows k+b .. k+np-1 are new
      const int r0 = k + b, r1 = k + np;
      for (int64_t e = threadIdx.x; e < static_cast<int64_t>(max(0, r1 - r0)) * w; e += blockDim.x) {
        const int r = r0 + static_cast<int>(e / w), c = static_cast<int>(e % w);
        rowp(r)[c] = G[static_cast<int64_t>(r) * w + c];
      }
      lds_barrier();
    }
    if (np > kPanelRowsPerThread * static_cast<int>(blockDim.x)) {
      // wider panels: eliminate in LDS (the rows do not fit the registers)
      for (int e = threadIdx.x; e < np * kPanel; e += blockDim.x) {
        const int ii = e / kPanel, c = e % kPanel, t = ii - c;
        P[ii * PS + c] = (c < nb && t >= 0 && t <= b) ? rowp(k + ii)[b - t] : TC(0);
      }
      lds_barrier();
      for (int c = 0; c < nb; ++c) {
        const TC d = P[c * PS + c];
        if (!(d > TC(0))) bad = true;
        const TC rd = TC(1) / d;
        for (int ii = c + 1 + threadIdx.x; ii < np; ii += blockDim.x) {
          const TC l = P[ii * PS + c] * rd;
          const int cend = min(nb, ii + 1);
          for (int c2 = c + 1; c2 < cend; ++c2) P[ii * PS + c2] -= l * P[c2 * PS + c];
        }
        lds_barrier();
      }
    } else {
    // eliminate the panel's columns with its rows in registers (thread t
    // owns rows t and t + blockDim.x); at step c the owners of rows c..nb-1
    // publish their column-c entries (double-buffered, one barrier a step)
    TC pr[kPanelRowsPerThread][kPanel];
#pragma clang loop unroll(full)
    for (int h2 = 0; h2 < kPanelRowsPerThread; ++h2) {
      const int ii = threadIdx.x + h2 * blockDim.x;
#pragma clang loop unroll(full)
      for (int c = 0; c < kPanel; ++c) {
        const int t = ii - c;
        pr[h2][c] = (ii < np && c < nb && t >= 0 && t <= b) ? rowp(k + ii)[b - t] : TC(0);
      }
    }
#pragma clang loop unroll(full)
    for (int c = 0; c < kPanel; ++c) {
      if (c < nb) {
        TC* cb = colbuf + (c & 1) * kPanel;
        if (static_cast<int>(threadIdx.x) >= c && static_cast<int>(threadIdx.x) < nb)
          cb[threadIdx.x] = pr[0][c];
        lds_barrier();
        const TC d = cb[c];
        if (!(d > TC(0))) bad = true;
        const TC rd = TC(1) / d;
#pragma clang loop unroll(full)
        for (int h2 = 0; h2 < kPanelRowsPerThread; ++h2) {
          const int ii = threadIdx.x + h2 * blockDim.x;
          if (ii > c && ii < np) {
            const TC l = pr[h2][c] * rd;
#pragma clang loop unroll(full)
            for (int c2 = c + 1; c2 < kPanel; ++c2)
              if (c2 < nb && c2 <= ii) pr[h2][c2] -= l * cb[c2];
          }
        }
      }
    }
#pragma clang loop unroll(full)
    for (int h2 = 0; h2 < kPanelRowsPerThread; ++h2) {
      const int ii = threadIdx.x + h2 * blockDim.x;
      if (ii < np) {
#pragma clang loop unroll(full)
        for (int c = 0; c < kPanel; ++c) P[ii * PS + c] = pr[h2][c];
      }
    }
    lds_barrier();
    }
    // D and unit-lower L of the panel's columns; Q for the trailing update
    for (int e = threadIdx.x; e < np * kPanel; e += blockDim.x) {
      const int ii = e / kPanel, c = e % kPanel, t = ii - c;
      const bool in = c < nb && t >= 0 && t <= b;
      const TC v = in ? (t == 0 ? P[c * PS + c] : P[ii * PS + c] / P[c * PS + c]) : TC(0);
      if (in) rowp(k + ii)[b - t] = v;
      if (ii >= nb) Q[c * mrow + ii] = v;
    }
    lds_barrier();
    // trailing update: A(k+ii, k+jj) -= sum_c P[ii][c] Q[c][jj], nb <= jj <= ii < np
    for (int ii = nb + wave; ii < np; ii += nwaves) {
      const TC* p = P + ii * PS;        // the same LDS address in every lane
      TC* row = rowp(k + ii) + b - ii;  // row[jj] = A(k+ii, k+jj)
      for (int j0 = nb; j0 <= ii; j0 += 256) {
        TC a[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int jj = j0 + lane + 64 * q;
          a[q] = jj <= ii ? row[jj] : TC(0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int jj = j0 + lane + 64 * q;
          if (jj <= ii) {
            TC acc = a[q];
#pragma unroll
            for (int c = 0; c < kPanel; ++c) acc -= p[c] * Q[c * mrow + jj];
            row[jj] = acc;
          }
        }
      }
    }
    if constexpr (kRing) lds_barrier(); else __syncthreads();  // global trailing rows
    if constexpr (kRing) {  // rows k .. k+nb-1 are final
      for (int64_t e = threadIdx.x; e < static_cast<int64_t>(nb) * w; e += blockDim.x) {
        const int r = k + static_cast<int>(e / w), c = static_cast<int>(e % w);
        G[static_cast<int64_t>(r) * w + c] = rowp(r)[c];
      }
      lds_barrier();
    }
  }
  __syncthreads();  // the factor rows in G are read by other threads next
  return bad;
}

// X <- A^{-1} X with A = L D L^T, by blocks of kSubRows rows.  Forward
// (z = L^-1 x), block [i0, i0+8): the entries L(i0+r, k), k in [i0-b, i0+8),
// are staged transposed in LDS (T[k-i0+b][r]); each thread owns whole columns
// of X, accumulates the coupling to the b rows before the block in registers
// (each X load feeds 8 multiply-adds) and then eliminates the block's own
// triangle.  Backward (x = D^-1 z - L^T x) mirrors it with T[j][r] =
// L(i0+j, i0+r).  Columns are independent, so the only barriers guard T.
// S: band_subst_elems(b) entries of LDS.
template <class TC, class TX>
__device__ void band_substitute(const TC* B, int n, int b, TX* X, int nck, TC* S) {
  constexpr int R = kSubRows;
  const int w = b + 1, nj = b + R;
  TC* T = S;
  TC* Dg = S + static_cast<int64_t>(nj) * R;
  for (int i0 = 0; i0 < n; i0 += R) {
    const int nr = min(R, n - i0);
    lds_barrier();
    for (int e = threadIdx.x; e < nj * R; e += blockDim.x) {
      const int j = e / R, r = e % R;
      const int k = i0 - b + j, t = b + r - j;  // L(i0+r, k)
      T[e] = (r < nr && k >= 0 && t >= 1 && t <= b) ? B[static_cast<int64_t>(i0 + r) * w + b - t] : TC(0);
    }
    lds_barrier();
    const int jb = max(0, b - i0);
    for (int c = threadIdx.x; c < nck; c += blockDim.x) {
      TC acc[R];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = TC(0);
      const TX* xc = X + static_cast<int64_t>(i0 - b) * nck + c;
#pragma unroll 4
      for (int j = jb; j < b; ++j) {
        const TC x = static_cast<TC>(xc[static_cast<int64_t>(j) * nck]);
        const TC* tj = T + j * R;
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] += tj[r] * x;
      }
      TC xv[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        TC a = r < nr ? static_cast<TC>(X[static_cast<int64_t>(i0 + r) * nck + c]) - acc[r] : TC(0);
#pragma unroll
        for (int q = 0; q < r; ++q) a -= T[(b + q) * R + r] * xv[q];
        xv[r] = a;
      }
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (r < nr) X[static_cast<int64_t>(i0 + r) * nck + c] = static_cast<TX>(xv[r]);
    }
  }
  const int nblk = (n + R - 1) / R;
  for (int blk = nblk - 1; blk >= 0; --blk) {
    const int i0 = blk * R, nr = min(R, n - i0);
    lds_barrier();
    for (int e = threadIdx.x; e < nj * R; e += blockDim.x) {
      const int j = e / R, r = e % R;
      const int i = i0 + j, t = j - r;  // L(i0+j, i0+r)
      T[e] = (r < nr && i < n && t >= 1 && t <= b) ? B[static_cast<int64_t>(i) * w + b - t] : TC(0);
    }
    if (threadIdx.x < R)
      Dg[threadIdx.x] = static_cast<int>(threadIdx.x) < nr ? B[static_cast<int64_t>(i0 + threadIdx.x) * w + b] : TC(1);
    lds_barrier();
    const int je = min(nj, n - i0);
    for (int c = threadIdx.x; c < nck; c += blockDim.x) {
      TC acc[R];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = TC(0);
      const TX* xc = X + static_cast<int64_t>(i0) * nck + c;
#pragma unroll 4
      for (int j = R; j < je; ++j) {
        const TC x = static_cast<TC>(xc[static_cast<int64_t>(j) * nck]);
        const TC* tj = T + j * R;
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] += tj[r] * x;
      }
      TC xv[R];
#pragma unroll
      for (int r = R - 1; r >= 0; --r) {
        TC a = r < nr ? static_cast<TC>(X[static_cast<int64_t>(i0 + r) * nck + c]) / Dg[r] - acc[r] : TC(0);
#pragma unroll
        for (int q = r + 1; q < R; ++q) a -= T[q * R + r] * xv[q];
        xv[r] = a;
      }
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (r < nr) X[static_cast<int64_t>(i0 + r) * nck + c] = static_cast<TX>(xv[r]);
    }
  }
  __syncthreads();
}

// Factorise and solve.  mode: band_mode(); B: the band, in LDS for mode 0,
// else in global memory; lds: LDS scratch of band_lds_elems(mode, n, b)
// entries (for mode 0 the band itself is its first n*(b+1) entries).
// `ticks` (optional): wall-clock stamps after factorisation, normalisation
// and substitution.
template <class TC, class TX>
__device__ bool band_ldlt_solve(int mode, TC* B, int n, int b, TX* X, int nck, TC* lds,
                                unsigned long long* ticks = nullptr) {
  bool bad;
  TC* S = lds;
  if (mode == 0) {
    bad = band_factor_inplace<TC>(B, n, b);
    if (ticks && threadIdx.x == 0) ticks[0] = wall_clock64();
    band_normalise<TC>(B, n, b);
    S = lds + static_cast<int64_t>(n) * (b + 1);
  } else {
    bad = mode == 1 ? band_factor_blocked<TC, true>(B, n, b, lds) : band_factor_blocked<TC, false>(B, n, b, lds);
    if (ticks && threadIdx.x == 0) ticks[0] = wall_clock64();
  }
  if (ticks && threadIdx.x == 0) ticks[1] = wall_clock64();
  band_substitute<TC, TX>(B, n, b, X, nck, S);
  if (ticks && threadIdx.x == 0) ticks[2] = wall_clock64();
  return bad;
}

}  // namespace fams
