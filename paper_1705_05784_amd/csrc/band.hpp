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
// Blocked modes also write the factor's columns contiguously (Lt, the lower
// band column by column) for the forward substitution.
// Substitution: band_solve_waves (band_substitute for bandwidths beyond it).
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
__device__ bool band_factor_blocked(TC* G, TC* Lt, int n, int b, TC* lds) {
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
    // D and unit-lower L of the panel's columns (also column by column
    // into Lt: Lt[j*(b+1) + t] = L(j+t, j)); Q for the trailing update
    for (int e = threadIdx.x; e < np * kPanel; e += blockDim.x) {
      const int c = e / np, ii = e % np, t = ii - c;
      const bool in = c < nb && t >= 0 && t <= b;
      const TC v = in ? (t == 0 ? P[c * PS + c] : P[ii * PS + c] / P[c * PS + c]) : TC(0);
      if (in) rowp(k + ii)[b - t] = v;
      if (in && t > 0) Lt[static_cast<int64_t>(k + c) * w + t] = v;
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

// ---- substitution by wavefronts --------------------------------------------
// One wavefront solves a group of NC columns of X with A = L D L^T, right-
// looking: lane l holds, in acc[.][s], the partial result of row
// 64 (c + s) + l (c the current chunk of 64 rows, s < M), so the window of M
// chunks covers every row one step can reach when 64 (M - 1) >= b.  Step k
// broadcasts the finished entry k (a readlane from chunk slot 0) and subtracts
// its multiple from the rows of the window it couples to; when a chunk is
// done its rows are stored and the window moves by one chunk.  Forward
// (z = L^-1 x) reads column k of L, backward (x = D^-1 z - L^T x) row k; the
// next 8 steps' entries are loaded while the current 8 are applied.  No
// barriers: columns are independent and B is read-only here.
//   column k of L: Fw[k*(b+1) + t*fstride + fbase], t = 1..b (row k + t)
//   row k of L:    Bw[k*(b+1) + b - t], t = 1..b (column k - t); D_k at t = 0
template <class TC>
__device__ __forceinline__ TC wave_bcast(TC v, int src) {
  if constexpr (sizeof(TC) == 4) {
    return __builtin_bit_cast(TC, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
  } else {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = static_cast<unsigned>(
        __builtin_amdgcn_readlane(static_cast<int>(static_cast<unsigned>(u)), src));
    const unsigned hi = static_cast<unsigned>(
        __builtin_amdgcn_readlane(static_cast<int>(static_cast<unsigned>(u >> 32)), src));
    return __builtin_bit_cast(TC, (static_cast<unsigned long long>(hi) << 32) | lo);
  }
}

template <class TC, class TX, class TO, int M, int NC, int J>
__device__ __forceinline__ void band_wave_columns(const TC* Bw, const TC* Fw, int fstride,
                                                  int fbase, int n, int b, TX* X, int nck,
                                                  int col, TO* Y) {
  static_assert(64 % J == 0 && (64 / J) % 2 == 0, "J steps per prefetch group");
  constexpr int GPC = 64 / J;  // prefetch groups per chunk
  const int lane = threadIdx.x & 63;
  const int w = b + 1;
  const int nch = (n + 63) >> 6;
  const int ng = nch * GPC;  // even
  TC acc[NC][M];
  TC bufA[J][M], bufB[J][M];
  auto xload = [&](int r, int j) -> TC {
    return (r >= 0 && r < n) ? static_cast<TC>(X[static_cast<int64_t>(r) * nck + col + j]) : TC(0);
  };
  auto step = [&](const TC (&buf)[J][M], int g, bool down) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int kk = down ? 63 - ((g % GPC) * J + j) : (g % GPC) * J + j;
      TC z[NC];
#pragma unroll
      for (int q = 0; q < NC; ++q) z[q] = wave_bcast(acc[q][0], kk);
#pragma unroll
      for (int s2 = 0; s2 < M; ++s2)
#pragma unroll
        for (int q = 0; q < NC; ++q) acc[q][s2] -= buf[j][s2] * z[q];
    }
  };

  // forward: chunk c = g / GPC, step k = J g + j, slot rows 64 (c + s) + lane
  auto fload = [&](TC (&buf)[J][M], int g) {
    const int c = g / GPC;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int k = g * J + j;
#pragma unroll
      for (int s2 = 0; s2 < M; ++s2) {
        const int r = 64 * (c + s2) + lane, t = r - k;
        const bool ok = t >= 1 && t <= b && r < n;
        const int idx = ok ? k * w + t * fstride + fbase : 0;
        const TC v = Fw[idx];
        buf[j][s2] = ok ? v : TC(0);
      }
    }
  };
#pragma unroll
  for (int s2 = 0; s2 < M; ++s2)
#pragma unroll
    for (int q = 0; q < NC; ++q) acc[q][s2] = xload(64 * s2 + lane, q);
  fload(bufA, 0);
  for (int g = 0; g < ng; g += 2) {
    fload(bufB, g + 1);
    step(bufA, g, false);
    fload(bufA, g + 2 < ng ? g + 2 : g);
    step(bufB, g + 1, false);
    if ((g + 1) % GPC == GPC - 1) {  // chunk (g+1)/GPC done
      const int c = (g + 1) / GPC, r = 64 * c + lane;
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        if (r < n) X[static_cast<int64_t>(r) * nck + col + q] = static_cast<TX>(acc[q][0]);
#pragma unroll
        for (int s2 = 0; s2 + 1 < M; ++s2) acc[q][s2] = acc[q][s2 + 1];
        acc[q][M - 1] = xload(64 * (c + M) + lane, q);
      }
    }
  }

  // backward: chunk c = nch-1 - g/GPC, steps k = 64 c + 63 - (J (g%GPC) + j),
  // slot rows 64 (c - s) + lane; rows enter scaled by 1/D; results go to Y
  auto entry = [&](int r, int q) -> TC {
    const TC d = (r >= 0 && r < n) ? Bw[r * w + b] : TC(1);
    return xload(r, q) / d;
  };
  auto bload = [&](TC (&buf)[J][M], int g) {
    const int c = nch - 1 - g / GPC;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int k = 64 * c + 63 - ((g % GPC) * J + j);
#pragma unroll
      for (int s2 = 0; s2 < M; ++s2) {
        const int r = 64 * (c - s2) + lane, t = k - r;
        const bool ok = t >= 1 && t <= b && r >= 0 && k < n;
        const int idx = ok ? k * w + b - t : 0;
        const TC v = Bw[idx];
        buf[j][s2] = ok ? v : TC(0);
      }
    }
  };
#pragma unroll
  for (int s2 = 0; s2 < M; ++s2)
#pragma unroll
    for (int q = 0; q < NC; ++q) acc[q][s2] = entry(64 * (nch - 1 - s2) + lane, q);
  bload(bufA, 0);
  for (int g = 0; g < ng; g += 2) {
    bload(bufB, g + 1);
    step(bufA, g, true);
    bload(bufA, g + 2 < ng ? g + 2 : g);
    step(bufB, g + 1, true);
    if ((g + 1) % GPC == GPC - 1) {
      const int c = nch - 1 - (g + 1) / GPC, r = 64 * c + lane;
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        if (r < n) Y[static_cast<int64_t>(r) * nck + col + q] = static_cast<TO>(acc[q][0]);
#pragma unroll
        for (int s2 = 0; s2 + 1 < M; ++s2) acc[q][s2] = acc[q][s2 + 1];
        acc[q][M - 1] = entry(64 * (c - M) + lane, q);
      }
    }
  }
}

// chunk slots for bandwidth b (64 (M - 1) >= b), 0 if beyond kWaveMaxBand
constexpr int kWaveMaxBand = 512;
__host__ __device__ inline int band_wave_slots(int b) {
  const int m = (b + 63) / 64 + 1;
  return b > kWaveMaxBand ? 0 : (m < 2 ? 2 : m);
}
// the instantiated slot counts: band_wave_slots rounded up to one of them
__host__ __device__ inline int band_wave_class(int b) {
  const int m = band_wave_slots(b);
  return m == 0 ? 0 : m <= 7 ? m : 9;
}

// single columns round-robin over the workgroup's waves (in-kernel use)
template <class TC, class TX, int M, int J>
__device__ void band_waves_single(const TC* Bw, const TC* Fw, int fstride, int fbase, int n,
                                  int b, TX* X, int nck) {
  const int wave = threadIdx.x / 64, nwaves = blockDim.x / 64;
  for (int q = wave; q < nck; q += nwaves)
    band_wave_columns<TC, TX, TX, M, 1, J>(Bw, Fw, fstride, fbase, n, b, X, nck, q, X);
}

// X <- A^{-1} X, one column per wavefront; false (nothing done) if b is
// beyond kWaveMaxBand.  Ends with a workgroup barrier.
template <class TC, class TX>
__device__ bool band_solve_waves(const TC* Bw, const TC* Fw, int fstride, int fbase, int n,
                                 int b, TX* X, int nck) {
  constexpr int J = sizeof(TC) == 4 ? 8 : 4;
  switch (band_wave_class(b)) {
    case 2: band_waves_single<TC, TX, 2, J>(Bw, Fw, fstride, fbase, n, b, X, nck); break;
    case 3: band_waves_single<TC, TX, 3, J>(Bw, Fw, fstride, fbase, n, b, X, nck); break;
    case 4: band_waves_single<TC, TX, 4, J>(Bw, Fw, fstride, fbase, n, b, X, nck); break;
    case 5: band_waves_single<TC, TX, 5, J>(Bw, Fw, fstride, fbase, n, b, X, nck); break;
    case 6: band_waves_single<TC, TX, 6, J>(Bw, Fw, fstride, fbase, n, b, X, nck); break;
    case 7: band_waves_single<TC, TX, 7, J>(Bw, Fw, fstride, fbase, n, b, X, nck); break;
    case 9: band_waves_single<TC, TX, 9, J>(Bw, Fw, fstride, fbase, n, b, X, nck); break;
    default: return false;
  }
  __syncthreads();
  return true;
}

// copy a factored band from LDS (mode 0) to global memory: the band as is
// into G and its columns into Lt (Lt[k*(b+1) + t] = L(k+t, k))
template <class TC>
__device__ void band_export(const TC* lds, TC* G, TC* Lt, int n, int b) {
  const int w = b + 1;
  for (int64_t e = threadIdx.x; e < static_cast<int64_t>(n) * w; e += blockDim.x) {
    G[e] = lds[e];
    const int k = static_cast<int>(e / w), t = static_cast<int>(e % w);
    Lt[e] = (t >= 1 && k + t < n) ? lds[static_cast<int64_t>(k + t) * w + b - t] : TC(0);
  }
}

// Factorise.  mode: band_mode(); mode 0: the band is the first n*(b+1)
// entries of lds; modes 1/2: the band is G (global memory) and Lt (n*(b+1)
// entries of global memory) receives L column by column; lds: LDS scratch of
// band_lds_elems(mode, n, b) entries.  `ticks` (optional): wall-clock stamps
// after factorisation and normalisation.
template <class TC>
__device__ bool band_factor(int mode, TC* G, TC* Lt, int n, int b, TC* lds,
                            unsigned long long* ticks = nullptr) {
  bool bad;
  if (mode == 0) {
    bad = band_factor_inplace<TC>(lds, n, b);
    if (ticks && threadIdx.x == 0) ticks[0] = wall_clock64();
    band_normalise<TC>(lds, n, b);
  } else {
    bad = mode == 1 ? band_factor_blocked<TC, true>(G, Lt, n, b, lds)
                    : band_factor_blocked<TC, false>(G, Lt, n, b, lds);
    if (ticks && threadIdx.x == 0) ticks[0] = wall_clock64();
  }
  if (ticks && threadIdx.x == 0) ticks[1] = wall_clock64();
  return bad;
}

// X <- A^{-1} X with the factor of band_factor (same mode, G, Lt, lds).
// Ends with a workgroup barrier.
template <class TC, class TX>
__device__ void band_solve(int mode, const TC* G, const TC* Lt, int n, int b, TX* X, int nck,
                           TC* lds) {
  if (mode == 0) {
    if (!band_solve_waves<TC, TX>(lds, lds, b, b, n, b, X, nck))
      band_substitute<TC, TX>(lds, n, b, X, nck, lds + static_cast<int64_t>(n) * (b + 1));
  } else {
    if (!band_solve_waves<TC, TX>(G, Lt, 1, 0, n, b, X, nck))
      band_substitute<TC, TX>(G, n, b, X, nck, lds);
  }
}

}  // namespace fams
