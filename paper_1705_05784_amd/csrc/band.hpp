// Banded LDL^T factorisation and solve.
//
// Storage: the lower band of a symmetric matrix of n rows and bandwidth b,
// row l, column l-t (0 <= t <= b) at B[l*(b+1) + b - t].  X holds nck
// right-hand sides, row-major [n][nck].  After factorisation the diagonal
// holds D and the entries below it the unit-lower L; Lt holds L column by
// column (Lt[j*(b+1) + t] = L(j+t, j), t >= 1) for the forward substitution.
//
// The factorisation (one workgroup) is blocked by kPanel columns.  The band
// lives in one of three places (band_mode):
//   0  LDS, after the panel scratch;
//   1  global memory, with a ring of b + kPanel band rows in LDS -- each row
//      is read once when a panel first reaches it and written once when final;
//   2  global memory, updated in place.
// Panel [k, k+nb): wavefront 0 factors the nb x nb diagonal block in
// registers (readlane broadcasts, no barriers); after one barrier each
// thread eliminates the panel columns of its own rows below the block
// against it and writes D, L, Lt and the trailing-update operands P
// (unscaled columns) and Q (scaled, transposed); the trailing update then
// subtracts the panel's rank-nb product from the triangle of the next b
// rows, lanes over columns (their nb entries of Q held in registers) and
// wavefronts over batches of rows, each batch's loads issued one batch ahead.
// Substitution: band_wave_columns (band_substitute for bandwidths beyond it).
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

// value of lane `src` (uniform) in every lane
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

constexpr int kPanel = 16;     // columns per panel of the blocked factorisation
constexpr int kSubRows = 8;    // rows per block of band_substitute
constexpr int kTrailRows = 8;  // rows per wavefront batch of the trailing update

// panel scratch: P, Q and the factored diagonal block (entries and 1/D)
__host__ __device__ inline int64_t band_panel_elems(int b) {
  return static_cast<int64_t>(kPanel + b) * (kPanel + 1) + static_cast<int64_t>(kPanel) * (kPanel + b) +
         kPanel * kPanel + kPanel;
}
__host__ __device__ inline int64_t band_ring_elems(int b) {
  return static_cast<int64_t>(kPanel + b) * (b + 1);
}
__host__ __device__ inline int64_t band_subst_elems(int b) {  // <= band_panel_elems(b)
  return static_cast<int64_t>(b + kSubRows) * kSubRows + kSubRows;
}

// storage mode for a band of n rows and bandwidth b with `lds` elements of
// LDS available; -1 if none fits
__host__ __device__ inline int band_mode(int n, int b, int64_t lds) {
  const int64_t pan = band_panel_elems(b);
  if (pan + static_cast<int64_t>(n) * (b + 1) <= lds) return 0;
  if (pan + band_ring_elems(b) <= lds) return 1;
  if (pan <= lds) return 2;
  return -1;
}
// LDS elements that mode `mode` uses: the panel scratch, then (mode 0) the
// band or (mode 1) the ring
__host__ __device__ inline int64_t band_lds_elems(int mode, int n, int b) {
  const int64_t pan = band_panel_elems(b);
  if (mode == 0) return pan + static_cast<int64_t>(n) * (b + 1);
  if (mode == 1) return pan + band_ring_elems(b);
  return pan;
}

// Blocked factorisation (see the top of this file).  kMode: band_mode();
// G: the band in global memory (modes 1, 2); lds: band_lds_elems() entries,
// the band itself at lds + band_panel_elems(b) in mode 0.  LDS layout: the
// panel P [(kPanel + b) rows][kPanel + 1] (unscaled columns), Q [kPanel]
// [kPanel + b] (Q[c][i] = L(k+i, k+c)), the diagonal block, then the band
// or the ring (row r in slot r mod (b + kPanel)).
// ph (optional): summed wall-clock ticks of the phases (ring load, panel,
// -, trailing update, ring store), by thread 0.
template <class TC, int kMode>
__device__ __forceinline__ bool band_factor_blocked(TC* G, TC* Lt, int n, int b, TC* lds,
                                    unsigned long long* ph = nullptr) {
  unsigned long long tph = (ph && threadIdx.x == 0) ? wall_clock64() : 0;
  auto mark = [&](int q) {
    if (ph && threadIdx.x == 0) {
      const unsigned long long t2 = wall_clock64();
      ph[q] += t2 - tph;
      tph = t2;
    }
  };
  const int w = b + 1;
  constexpr int PS = kPanel + 1;
  const int mrow = kPanel + b;
  TC* P = lds;
  TC* Q = P + static_cast<int64_t>(mrow) * PS;
  TC* dgu = Q + static_cast<int64_t>(kPanel) * mrow;  // diagonal block: u(i, c) at [i * kPanel + c], c < i
  TC* dgr = dgu + kPanel * kPanel;                     // 1 / d_c
  TC* band = dgr + kPanel;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, nwaves = blockDim.x / 64;
  auto rowp = [&](int r) -> TC* {  // band row r
    if constexpr (kMode == 0) return band + static_cast<int64_t>(r) * w;
    else if constexpr (kMode == 1) return band + static_cast<int64_t>(r % mrow) * w;
    else return G + static_cast<int64_t>(r) * w;
  };
  bool bad = false;
  if constexpr (kMode == 1) {  // rows 0..b-1 enter before the first panel
    for (int64_t e = tid; e < static_cast<int64_t>(min(n, b)) * w; e += blockDim.x)
      band[e] = G[e];
  }
  for (int k = 0; k < n; k += kPanel) {
    const int nb = min(kPanel, n - k);
    const int np = min(n - k, nb + b);  // panel rows k .. k+np-1
    const int s0 = kMode == 1 ? k % mrow : 0;
    auto prow = [&](int ii) -> TC* {  // band row k + ii, 0 <= ii < np
      if constexpr (kMode == 1) {
        int sl = s0 + ii;
        sl -= sl >= mrow ? mrow : 0;
        return band + static_cast<int64_t>(sl) * w;
      } else {
        return rowp(k + ii);
      }
    };
    if constexpr (kMode == 1) {  // rows k+b .. k+np-1 are new
      const int r0 = k + b, r1 = k + np;
      for (int64_t e = tid; e < static_cast<int64_t>(max(0, r1 - r0)) * w; e += blockDim.x) {
        const int r = r0 + static_cast<int>(e / w), c = static_cast<int>(e % w);
        rowp(r)[c] = G[static_cast<int64_t>(r) * w + c];
      }
      lds_barrier();
    }
    mark(0);
    // diagonal block: lane i < nb of wavefront 0 holds row k+i, columns
    // k..k+i; rows and columns nb..kPanel-1 are padded with the identity
    // (which the steps keep exact) so that all kPanel steps run without
    // branches; entries above the diagonal are scratch and never read
    if (wave == 0) {
      TC r[kPanel];
      const bool own = lane < nb;
      const TC* rw = prow(own ? lane : 0);
#pragma unroll
      for (int c = 0; c < kPanel; ++c) {
        const int t = lane - c;
        r[c] = (own && c < nb && t >= 0 && t <= b) ? rw[b - t] : (lane == c ? TC(1) : TC(0));
      }
#pragma unroll
      for (int c = 0; c < kPanel; ++c) {
        const TC d = wave_bcast(r[c], c);  // u(c, c) = d_c
        if (c < nb && !(d > TC(0))) bad = true;
        const TC rd = TC(1) / d;
        const TC l = r[c] * rd;
        if (lane == c) dgr[c] = rd;
#pragma unroll
        for (int c2 = c + 1; c2 < kPanel; ++c2) r[c2] -= l * wave_bcast(r[c], c2);  // u(c2, c)
        __builtin_amdgcn_sched_barrier(0);
      }
      if (lane < kPanel) {
#pragma unroll
        for (int c = 0; c < kPanel; ++c) {
          if (c < lane) dgu[lane * kPanel + c] = r[c];
          if (own && c <= lane) P[lane * PS + c] = r[c];
        }
      }
    }
    lds_barrier();
    // rows below the diagonal block: eliminate the panel columns against it
    // (unscaled results to P)
    for (int ii = nb + tid; ii < np; ii += blockDim.x) {
      const TC* rw = prow(ii);
      TC x[kPanel];
#pragma unroll
      for (int c = 0; c < kPanel; ++c) {
        const int t = ii - c;
        x[c] = (c < nb && t <= b) ? rw[b - t] : TC(0);
      }
#pragma unroll
      for (int c = 0; c < kPanel; ++c) {
        const TC l = x[c] * dgr[c];
#pragma unroll
        for (int c2 = c + 1; c2 < kPanel; ++c2) x[c2] -= l * dgu[c2 * kPanel + c];
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int c = 0; c < kPanel; ++c) P[ii * PS + c] = x[c];
    }
    lds_barrier();
    mark(1);
    // D and unit-lower L of the panel's columns into the band and (column
    // by column) Lt; Q for the trailing update
    for (int e = tid; e < np * kPanel; e += blockDim.x) {
      const int c = e / np, ii = e % np, t = ii - c;
      const bool in = c < nb && t >= 0 && t <= b;
      const TC u = P[ii * PS + c];
      const TC v = in ? (t == 0 ? u : u * dgr[c]) : TC(0);
      if (in) {
        prow(ii)[b - t] = v;
        if (t > 0) Lt[static_cast<int64_t>(k + c) * w + t] = v;
      }
      if (ii >= nb) Q[c * mrow + ii] = v;
    }
    lds_barrier();
    mark(2);
    // trailing update: A(k+ii, k+jj) -= sum_c P[ii][c] Q[c][jj], nb <= jj <= ii < np
    for (int j0 = nb; j0 < np; j0 += 64) {
      const int jj = j0 + lane;
      TC qv[kPanel];
#pragma unroll
      for (int c = 0; c < kPanel; ++c) qv[c] = jj < np ? Q[c * mrow + jj] : TC(0);
      TC a[kTrailRows], an[kTrailRows];
      auto load = [&](TC (&dst)[kTrailRows], int i0) {
#pragma unroll
        for (int q = 0; q < kTrailRows; ++q) {
          const int ii = min(i0 + q, np - 1), jc = min(jj, ii);  // clamped, in the band
          dst[q] = prow(ii)[b - ii + jc];
        }
      };
      int i0 = j0 + wave * kTrailRows;
      load(a, i0);
      for (; i0 < np; i0 += nwaves * kTrailRows) {
        load(an, i0 + nwaves * kTrailRows);
#pragma unroll
        for (int q = 0; q < kTrailRows; ++q) {
          const int ii = i0 + q;
          if (ii < np) {
            const TC* p = P + ii * PS;
            TC acc = a[q];
#pragma unroll
            for (int c = 0; c < kPanel; ++c) acc -= p[c] * qv[c];
            if (jj <= ii) prow(ii)[b - ii + jj] = acc;
          }
          __builtin_amdgcn_sched_barrier(0);  // one row's P entries live at a time
        }
#pragma unroll
        for (int q = 0; q < kTrailRows; ++q) a[q] = an[q];
      }
    }
    if constexpr (kMode == 2) __syncthreads(); else lds_barrier();
    mark(3);
    if constexpr (kMode == 1) {  // rows k .. k+nb-1 are final
      for (int64_t e = tid; e < static_cast<int64_t>(nb) * w; e += blockDim.x) {
        const int r = k + static_cast<int>(e / w), c = static_cast<int>(e % w);
        G[static_cast<int64_t>(r) * w + c] = rowp(r)[c];
      }
      lds_barrier();
    }
    mark(4);
  }
  __syncthreads();  // the factor rows are read by other threads next
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

// copy a band factored in LDS (mode 0) to global memory
template <class TC>
__device__ void band_export(const TC* band_lds, TC* G, int n, int b) {
  for (int64_t e = threadIdx.x; e < static_cast<int64_t>(n) * (b + 1); e += blockDim.x)
    G[e] = band_lds[e];
}

// Factorise: mode = band_mode(); G, Lt in global memory (G unused in mode
// 0, whose band is at lds + band_panel_elems(b)); lds: band_lds_elems()
// entries.  `ticks` (optional): ticks[0], ticks[1] = wall clock when done,
// ticks[6..10] the phase sums of band_factor_blocked.
template <class TC>
__device__ bool band_factor(int mode, TC* G, TC* Lt, int n, int b, TC* lds,
                            unsigned long long* ticks = nullptr) {
  unsigned long long* ph = ticks ? ticks + 6 : nullptr;
  bool bad;
  if (mode == 0) bad = band_factor_blocked<TC, 0>(G, Lt, n, b, lds, ph);
  else if (mode == 1) bad = band_factor_blocked<TC, 1>(G, Lt, n, b, lds, ph);
  else bad = band_factor_blocked<TC, 2>(G, Lt, n, b, lds, ph);
  if (ticks && threadIdx.x == 0) ticks[0] = ticks[1] = wall_clock64();
  return bad;
}

}  // namespace fams
