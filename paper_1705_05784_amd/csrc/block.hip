// Several right-hand sides on one setup, iterated in lock-step.
//
// The paper builds the F-AMS operators once per pressure system and reuses
// them for every solve with that system (Sec. 4.6); Table 1's stage is linear
// in the residual, so K right-hand sides can share every pass over the
// operators.  Block vectors hold the K values of a row next to each other
// (x[i * K + r]): the fine operator, P, R, the ILU(0) factors and the dense
// A_c^{-1} are read once per stage for all K, and the K lanes of a row
// gather the same neighbours.  Each right-hand side keeps its own outer
// iteration (GMRES with its own Hessenberg matrix, Givens rotations, restart
// and stopping test, or the Table 1 loop): a right-hand side that has met its
// stopping test is masked out (its updates are multiplied by zero) while the
// others continue, so every column follows the same iteration as a solve of
// its own.  Right-hand sides are taken in groups of K in {2, 4, 8, 16}, as
// many as the device memory holds.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <type_traits>
#include <vector>

#include "internal.hpp"

namespace fams {
namespace {

constexpr int kT = 256;
constexpr int kRedBlocks = 2048;  // workgroups of the multi-dot passes

// ---- layout ------------------------------------------------------------------
// Q[i * K + r] = q[r * n + i] for r < nr, 0 for the padding lanes: a
// transpose through LDS, a tile of kPackRows rows per workgroup, so that both
// sides are read and written in contiguous runs
constexpr int kPackRows = 256;

template <int K>
__global__ void __launch_bounds__(256) k_pack(int n, int nr, const double* q, double* Q) {
  __shared__ double t[kPackRows * (K + 1)];  // row l at l (K + 1): padded against bank conflicts
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * kPackRows;
  for (int s = threadIdx.x; s < kPackRows * K; s += blockDim.x) {
    const int r = s / kPackRows, l = s % kPackRows;
    const int64_t i = i0 + l;
    t[l * (K + 1) + r] = (r < nr && i < n) ? q[static_cast<int64_t>(r) * n + i] : 0.0;
  }
  __syncthreads();
  for (int s = threadIdx.x; s < kPackRows * K; s += blockDim.x) {
    const int l = s / K, r = s % K;
    if (i0 + l < n) Q[(i0 + l) * K + r] = t[l * (K + 1) + r];
  }
}

template <int K>
__global__ void __launch_bounds__(256) k_unpack(int n, int nr, const double* Q, double* q) {
  __shared__ double t[kPackRows * (K + 1)];
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * kPackRows;
  for (int s = threadIdx.x; s < kPackRows * K; s += blockDim.x) {
    const int l = s / K, r = s % K;
    if (i0 + l < n) t[l * (K + 1) + r] = Q[(i0 + l) * K + r];
  }
  __syncthreads();
  for (int s = threadIdx.x; s < kPackRows * K; s += blockDim.x) {
    const int r = s / kPackRows, l = s % kPackRows;
    const int64_t i = i0 + l;
    if (r < nr && i < n) q[static_cast<int64_t>(r) * n + i] = t[l * (K + 1) + r];
  }
}

// ---- operators on block vectors ------------------------------------------------
// Row-wise kernels take their rows in XCD-contiguous ranges (xcd_block,
// xcd_grid), so the neighbours a row gathers (the previous and next rows,
// lines and planes) were mostly brought into the same XCD's L2 by its own
// earlier workgroups.

// Y = M X (kResid: Y = B - M X, B may be null or alias Y) on block vectors:
// K / 2 threads per row, each with two right-hand sides (r, r + 1) whose
// values of a neighbour it gathers in one load; the threads of a row read
// its entries at the same addresses
// two consecutive values of a block vector (right-hand sides r, r + 1; r even)
template <class T> struct Pair;
template <> struct Pair<double> { using V = double2; };
template <> struct Pair<float> { using V = float2; };

template <class T>
__device__ __forceinline__ void load_pair(const T* p, double& a, double& b) {
  const typename Pair<T>::V v = *reinterpret_cast<const typename Pair<T>::V*>(p);
  a = static_cast<double>(v.x);
  b = static_cast<double>(v.y);
}

template <class T>
__device__ __forceinline__ void store_pair_to(T* p, double a, double b) {
  typename Pair<T>::V v;
  v.x = static_cast<T>(a);
  v.y = static_cast<T>(b);
  *reinterpret_cast<typename Pair<T>::V*>(p) = v;
}

// The products with A and P in the lock-step solves read the matrix in a
// fixed-width form: kEll (column, value) slots per row in CSR order, padded
// with (a column of the row, 0), and per row the CSR position and count of
// the entries beyond kEll.  A row's slots sit at a position computed from
// the row alone, so the index and value loads need no row-pointer load
// before them: one dependent memory step less per row than CSR, and wide
// loads.  Same terms in the same order as the CSR product (padding adds +0).
constexpr int kEll = 8;

template <class TV>
__device__ __forceinline__ void load_ell_vals(const TV* p, TV* v);
template <>
__device__ __forceinline__ void load_ell_vals<double>(const double* p, double* v) {
#pragma unroll
  for (int k = 0; k < kEll; k += 2) {
    const double2 t = reinterpret_cast<const double2*>(p)[k / 2];
    v[k] = t.x;
    v[k + 1] = t.y;
  }
}
template <>
__device__ __forceinline__ void load_ell_vals<float>(const float* p, float* v) {
#pragma unroll
  for (int k = 0; k < kEll; k += 4) {
    const float4 t = reinterpret_cast<const float4*>(p)[k / 4];
    v[k] = t.x;
    v[k + 1] = t.y;
    v[k + 2] = t.z;
    v[k + 3] = t.w;
  }
}

template <class TV, class TX, class TB, class TY, int K, bool kResid>
__global__ void __launch_bounds__(256)
k_bspmv_ell(int n, const int* ecol, const TV* eval, const int* ovf, const int* ci, const TV* val,
            const TX* X, const TB* B, TY* Y, RowTiling tl) {
  constexpr int H = K / 2;
  const int64_t e2 = xcd_block() * blockDim.x + threadIdx.x;
  if (e2 >= static_cast<int64_t>(n) * H) return;
  const int i = tiled_row(tl, static_cast<int>(e2 / H)), r = 2 * static_cast<int>(e2 % H);
  const int64_t o = static_cast<int64_t>(i) * K + r;
  int c[kEll];
  TV v[kEll];
#pragma unroll
  for (int k = 0; k < kEll; k += 4) {
    const int4 t = reinterpret_cast<const int4*>(ecol + static_cast<int64_t>(i) * kEll)[k / 4];
    c[k] = t.x;
    c[k + 1] = t.y;
    c[k + 2] = t.z;
    c[k + 3] = t.w;
  }
  load_ell_vals<TV>(eval + static_cast<int64_t>(i) * kEll, v);
  const int2 ov = reinterpret_cast<const int2*>(ovf)[i];
  double b0 = 0.0, b1 = 0.0;
  if (kResid && B) load_pair<TB>(B + o, b0, b1);
  double x0[kEll], x1[kEll];
#pragma unroll
  for (int k = 0; k < kEll; ++k) load_pair<TX>(X + static_cast<int64_t>(c[k]) * K + r, x0[k], x1[k]);
  double s0 = 0.0, s1 = 0.0;
#pragma unroll
  for (int k = 0; k < kEll; ++k) {
    s0 += static_cast<double>(v[k]) * x0[k];
    s1 += static_cast<double>(v[k]) * x1[k];
  }
  for (int p = ov.x; p < ov.x + ov.y; ++p) {
    double a0, a1;
    load_pair<TX>(X + static_cast<int64_t>(ci[p]) * K + r, a0, a1);
    s0 += static_cast<double>(val[p]) * a0;
    s1 += static_cast<double>(val[p]) * a1;
  }
  if constexpr (kResid) {
    s0 = b0 - s0;
    s1 = b1 - s1;
  }
  store_pair_to<TY>(Y + o, s0, s1);
}

// columns and overflow ranges of the fixed-width form (one thread per row);
// a padding slot repeats the row's first column (column 0 for an empty row):
// a column of the matrix whatever its shape, and a gather already made
__global__ void k_ell_cols(int n, const int* rp, const int* ci, int* ecol, int* ovf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p0 = rp[i], d = rp[i + 1] - p0;
  const int pad = d > 0 ? ci[p0] : 0;
  for (int k = 0; k < kEll; ++k) ecol[static_cast<int64_t>(i) * kEll + k] = k < d ? ci[p0 + k] : pad;
  ovf[2 * i] = p0 + kEll;
  ovf[2 * i + 1] = d > kEll ? d - kEll : 0;
}

template <class TV>
__global__ void k_ell_vals(int n, const int* rp, const TV* val, TV* eval) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p0 = rp[i], d = rp[i + 1] - p0;
  for (int k = 0; k < kEll; ++k) eval[static_cast<int64_t>(i) * kEll + k] = k < d ? val[p0 + k] : TV(0);
}

// sum over the lanes of a workgroup of 256 that hold the same r = tid % K
// (fixed order: shuffles inside each wavefront, then the four wavefronts in
// order); the result is valid in threads 0..K-1
template <int K>
__device__ double group_sum(double v) {
  __shared__ double s[4][K];
  for (int o = 32; o >= K; o >>= 1) v += __shfl_down(v, o, 64);
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  __syncthreads();
  if (l < K) s[w][l] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x < K)
    for (int q = 0; q < 4; ++q) t += s[q][threadIdx.x];
  return t;
}

// sum over the lanes of a workgroup of 256 that share tid % (K/2), i.e. the
// same pair (2l, 2l + 1) of right-hand sides in the two-element kernels
// below; valid in threads 0 .. K/2 - 1
template <int K>
__device__ double pair_sum(double v) {
  constexpr int H = K / 2;
  __shared__ double s[4][H];
  for (int o = 32; o >= H; o >>= 1) v += __shfl_down(v, o, 64);
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  __syncthreads();
  if (l < H) s[w][l] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x < H)
    for (int q = 0; q < 4; ++q) t += s[q][threadIdx.x];
  return t;
}

// Y[row * K + r] = sum_p M[row, p] X[col_p * K + r] for the fat rows of R =
// P^T: one workgroup per row, 512 / K groups of K / 2 lanes (two right-hand
// sides each) stride over the row's entries, then a fixed-order sum across
// the groups
template <class TV, class TX, int K>
__global__ void __launch_bounds__(256)
k_brestrict(int nrows, const int* rp, const int* ci, const TV* val, const TX* X, double* Y) {
  constexpr int H = K / 2, G = 256 / H;
  const int row = blockIdx.x;
  const int r = 2 * (threadIdx.x % H), g = threadIdx.x / H;
  double s0 = 0.0, s1 = 0.0;
  const int p1 = rp[row + 1];
  for (int pb = rp[row] + g; pb < p1; pb += 4 * G) {
    int c[4];
    TV v[4];
    double x0[4], x1[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (pb + k * G < p1) {
        c[k] = ci[pb + k * G];
        v[k] = val[pb + k * G];
      }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (pb + k * G < p1) load_pair<TX>(X + static_cast<int64_t>(c[k]) * K + r, x0[k], x1[k]);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (pb + k * G < p1) {
        s0 += static_cast<double>(v[k]) * x0[k];
        s1 += static_cast<double>(v[k]) * x1[k];
      }
  }
  s0 = pair_sum<K>(s0);
  s1 = pair_sum<K>(s1);
  if (threadIdx.x < H) {
    Y[static_cast<int64_t>(row) * K + 2 * threadIdx.x] = s0;
    Y[static_cast<int64_t>(row) * K + 2 * threadIdx.x + 1] = s1;
  }
}

// coarse solve X = A_c^{-1} Y with the dense inverse (column-major nc x nc):
// a workgroup takes 256 rows and one chunk of `w` columns, stages the chunk's
// right-hand sides in LDS 64 columns at a time and keeps K sums per row in
// registers; partial results per chunk are added in chunk order afterwards
template <int K>
__global__ void __launch_bounds__(256)
k_bcoarse_part(int nc, int w, const double* M, const double* Y, double* part) {
  __shared__ double ys[64 * K];
  const int I = blockIdx.x * 256 + threadIdx.x;
  const int c0 = blockIdx.y * w, c1 = min(nc, c0 + w);
  double acc[K];
#pragma unroll
  for (int r = 0; r < K; ++r) acc[r] = 0.0;
  for (int cb = c0; cb < c1; cb += 64) {
    const int ce = min(64, c1 - cb);
    __syncthreads();
    for (int t = threadIdx.x; t < 64 * K; t += 256)
      ys[t] = t < ce * K ? Y[static_cast<int64_t>(cb) * K + t] : 0.0;
    __syncthreads();
    if (I < nc) {
      const double* col = M + static_cast<int64_t>(cb) * nc + I;
#pragma unroll 16
      for (int c = 0; c < ce; ++c) {
        const double a = col[static_cast<int64_t>(c) * nc];
#pragma unroll
        for (int r = 0; r < K; ++r) acc[r] += a * ys[c * K + r];
      }
    }
  }
  if (I < nc) {
    double* o = part + (static_cast<int64_t>(blockIdx.y) * nc + I) * K;
#pragma unroll
    for (int r = 0; r < K; ++r) o[r] = acc[r];
  }
}

// The same on FP64 MFMA for groups of 16 or more (K a multiple of 16): each
// wavefront forms 16 rows x K of the chunk's partial product with
// v_mfma_f64_16x16x4 (per instruction lane l supplies A[l%16][l/16] =
// M[row, col] and B[l/16][l%16] = Y[col, rhs]; accumulator element q holds
// D[4q + l/16][l%16]), its operands loaded straight from memory kBcU steps
// of four columns ahead.  One eight-byte operand per lane and 1024
// multiply-adds, where the vector form above reads one LDS value per
// multiply-add and lane.
typedef double v4d_b __attribute__((ext_vector_type(4)));
constexpr int kBcU = 4;

template <int K>
__global__ void __launch_bounds__(256)
k_bcoarse_mfma(int nc, int w, const double* M, const double* Y, double* part) {
  constexpr int NT = K / 16;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int I0 = (blockIdx.x * 4 + wave) * 16;
  if (I0 >= nc) return;  // a whole wavefront; the kernel has no barrier
  const int c0 = blockIdx.y * w, c1 = min(nc, c0 + w);
  const int i = I0 + lane % 16, kq = lane / 16, j = lane % 16;
  const bool row_ok = i < nc;
  v4d_b acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = v4d_b{0.0, 0.0, 0.0, 0.0};
  for (int c = c0; c < c1; c += 4 * kBcU) {
    double fa[kBcU], fb[kBcU][NT];
#pragma unroll
    for (int u = 0; u < kBcU; ++u) {
      const int col = c + 4 * u + kq;
      const bool ok = col < c1;
      fa[u] = (ok && row_ok) ? M[static_cast<int64_t>(col) * nc + i] : 0.0;
#pragma unroll
      for (int t = 0; t < NT; ++t) fb[u][t] = ok ? Y[static_cast<int64_t>(col) * K + t * 16 + j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kBcU; ++u)
#pragma unroll
      for (int t = 0; t < NT; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[u], fb[u][t], acc[t], 0, 0, 0);
  }
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = I0 + 4 * q + kq;
      if (row < nc) part[(static_cast<int64_t>(blockIdx.y) * nc + row) * K + t * 16 + j] = acc[t][q];
    }
}

__global__ void k_bcoarse_red(int64_t nk, int nch, const double* part, double* X) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nk) return;
  double s = 0.0;
  for (int c = 0; c < nch; ++c) s += part[static_cast<int64_t>(c) * nk + e];
  X[e] = s;
}

template <class TA, class TY>
__global__ void k_bcast(int64_t n, const TA* a, TY* y) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = static_cast<TY>(a[i]);
}

template <class TA, class TB, class TY>
__global__ void k_badd(int64_t n, const TA* a, const TB* b, TY* y) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = static_cast<TY>(static_cast<double>(a[i]) + static_cast<double>(b[i]));
}

// ---- reductions and Krylov updates per right-hand side ---------------------------
// part[(b * pstride + v) * K + r] = block b's share of sum_i V_v[i, r] w[i, r]
// for v < nv, in batches of kDotBatch vectors so that w is read once per batch
constexpr int kDotBatch = 8;

template <int K>
__device__ void store_dots(const double* acc, int nb, int v0, double* part, int pstride) {
#pragma unroll
  for (int u = 0; u < kDotBatch; ++u) {
    if (u >= nb) break;
    const double s = group_sum<K>(acc[u]);
    if (threadIdx.x < K)
      part[(static_cast<int64_t>(blockIdx.x) * pstride + v0 + u) * K + threadIdx.x] = s;
  }
}


// the streaming Krylov kernels take two consecutive entries per thread (one
// 16-byte load per vector; K is even, so both entries are of one row and of
// right-hand sides 2l and 2l + 1)
template <int K>
__device__ void store_pair(double s0, double s1, int v, double* part, int pstride) {
  s0 = pair_sum<K>(s0);
  s1 = pair_sum<K>(s1);
  if (threadIdx.x < K / 2) {
    double* o = part + (static_cast<int64_t>(blockIdx.x) * pstride + v) * K + 2 * threadIdx.x;
    o[0] = s0;
    o[1] = s1;
  }
}

template <int K>
__global__ void __launch_bounds__(256)
k_bmdot_part(int64_t nk, int nv, const double* V, int64_t ldv, const double* w, double* part,
             int pstride) {
  const int64_t n2 = nk / 2;
  const double2* w2 = reinterpret_cast<const double2*>(w);
  for (int v0 = 0; v0 < nv; v0 += kDotBatch) {
    const int nb = min(kDotBatch, nv - v0);
    double a0[kDotBatch], a1[kDotBatch];
#pragma unroll
    for (int u = 0; u < kDotBatch; ++u) a0[u] = a1[u] = 0.0;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < n2;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
      const double2 we = w2[e];
      // all loads of the batch unconditional (past nv they repeat the last
      // vector and their sums are dropped), so they issue back to back
#pragma unroll
      for (int u = 0; u < kDotBatch; ++u) {
        const double2 x =
            reinterpret_cast<const double2*>(V + static_cast<int64_t>(min(v0 + u, nv - 1)) * ldv)[e];
        a0[u] += x.x * we.x;
        a1[u] += x.y * we.y;
      }
    }
#pragma unroll
    for (int u = 0; u < kDotBatch; ++u) {
      if (u >= nb) break;
      store_pair<K>(a0[u], a1[u], v0 + u, part, pstride);
    }
  }
}

// The two streaming passes below read up to kFuseMax basis vectors per
// entry.  Every vector is addressed as a uniform base (scalar registers)
// plus one byte offset shared by all of them (a 32-bit vector register):
// left to itself, the compiler's loop strength reduction keeps one 64-bit
// pointer per vector in vector registers, and the register pressure then
// serialises the loads.  The empty asm statement hides the offset's
// induction from that transformation.  Usable while a block vector is
// under 4 GiB (checked on the host; larger ones take the general kernels).
constexpr int kFuseMax = 4 * kDotBatch;

// At most three waves per SIMD: lets the scheduler keep all of an entry's
// loads in flight at once instead of trading them for occupancy (three
// waves of 32 outstanding 16-byte loads per lane saturate HBM).
#define FAMS_STREAM_WAVES __attribute__((amdgpu_waves_per_eu(1, 3)))

__device__ __forceinline__ uint32_t opaque(uint32_t x) {
  asm volatile("" : "+v"(x));
  return x;
}

template <class T>
__device__ __forceinline__ T load_at(const char* base, uint32_t off) {
  return *reinterpret_cast<const T*>(base + off);
}

// the first Gram-Schmidt correction and the second pass's dots in one pass
// over the rows: w <- w - sum_v coef[r, v] V_v, then the partial dots of the
// new w with V_0..V_{nv-1}; each V value is loaded once and kept in a
// register between the two uses.  NV (a multiple of 4, nv <= NV <= kFuseMax)
// fixes the register arrays at compile time, so the NV loads of an entry are
// issued back to back with no branch between them: the vectors past nv
// repeat V_{nv-1} (cache hits) with a zero coefficient, which leaves the sum
// bit for bit what it is over nv vectors.  The grid stride is a multiple of
// 256, so a thread keeps one right-hand side r = threadIdx.x % K and reads
// its coefficients from LDS.
template <int K, int NV>
__global__ void __launch_bounds__(256) FAMS_STREAM_WAVES
k_bmaxpy_mdot(int64_t nk, int nv, const double* V, int64_t ldv, const double* coef, int cstride,
              double* w, double* part, int pstride) {
  __shared__ double cs[K * NV];
  for (int t = threadIdx.x; t < K * NV; t += blockDim.x) {
    const int r = t / NV, v = t % NV;
    cs[t] = v < nv ? coef[static_cast<int64_t>(r) * cstride + v] : 0.0;
  }
  __syncthreads();
  const double* c = cs + (threadIdx.x % K) * NV;
  const char* Vb = reinterpret_cast<const char*>(V);
  char* wb = reinterpret_cast<char*>(w);
  const int64_t ld8 = ldv * 8;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  const uint32_t end = static_cast<uint32_t>(nk * 8);
  const uint32_t step = gridDim.x * blockDim.x * 8u;
  for (uint32_t off0 = (blockIdx.x * blockDim.x + threadIdx.x) * 8u; off0 < end; off0 += step) {
    const uint32_t off = opaque(off0);
    double vv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) vv[v] = load_at<double>(Vb + ld8 * min(v, nv - 1), off);
    double s = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) s += c[v] * vv[v];
    const double we = load_at<double>(wb, off) - s;
    *reinterpret_cast<double*>(wb + off) = we;
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += vv[v] * we;
  }
#pragma unroll
  for (int a = 0; a < NV / kDotBatch + (NV % kDotBatch ? 1 : 0); ++a) {
    if (a * kDotBatch >= nv) break;
    double blk[kDotBatch];
#pragma unroll
    for (int u = 0; u < kDotBatch; ++u) blk[u] = a * kDotBatch + u < NV ? acc[a * kDotBatch + u] : 0.0;
    store_dots<K>(blk, min(kDotBatch, nv - a * kDotBatch), a * kDotBatch, part, pstride);
  }
}

// block vectors of nk entries: can the offset-addressed passes take them?
inline bool offset_addressable(int64_t nk, unsigned nb) {
  return (nk * 8 + static_cast<int64_t>(nb) * kT * 16) < (int64_t(1) << 32);
}

// launch of the fused pass with NV = nv rounded up to a multiple of 4
template <int K>
void launch_bmaxpy_mdot(Handle* h, unsigned nb, int64_t nk, int nv, const double* V, int64_t ldv,
                        const double* coef, int cstride, double* w, double* part, int pstride) {
#define FAMS_MDOT(NV)                                                                          \
  LAUNCH(h, "bmaxpy_mdot", (k_bmaxpy_mdot<K, NV>), nb, kT, 0, nk, nv, V, ldv, coef, cstride, w, \
         part, pstride)
  switch ((nv + 3) / 4) {
    case 1: FAMS_MDOT(4); break;
    case 2: FAMS_MDOT(8); break;
    case 3: FAMS_MDOT(12); break;
    case 4: FAMS_MDOT(16); break;
    case 5: FAMS_MDOT(20); break;
    case 6: FAMS_MDOT(24); break;
    case 7: FAMS_MDOT(28); break;
    case 8: FAMS_MDOT(32); break;
    default: FAMS_REQUIRE(false, FAMS_ERR_CAPACITY, "fused Gram-Schmidt pass: too many vectors");
  }
#undef FAMS_MDOT
}

// the multi-dot h = V^T w of the first Gram-Schmidt pass, one entry per
// thread with all NV loads in flight (as in the fused pass; vectors past nv
// repeat the last one and their sums are dropped)
template <int K, int NV>
__global__ void __launch_bounds__(256) FAMS_STREAM_WAVES
k_bmdot(int64_t nk, int nv, const double* V, int64_t ldv, const double* w, double* part,
        int pstride) {
  const char* Vb = reinterpret_cast<const char*>(V);
  const char* wb = reinterpret_cast<const char*>(w);
  const int64_t ld8 = ldv * 8;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  const uint32_t end = static_cast<uint32_t>(nk * 8);
  const uint32_t step = gridDim.x * blockDim.x * 8u;
  for (uint32_t off0 = (blockIdx.x * blockDim.x + threadIdx.x) * 8u; off0 < end; off0 += step) {
    const uint32_t off = opaque(off0);
    const double we = load_at<double>(wb, off);
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += load_at<double>(Vb + ld8 * min(v, nv - 1), off) * we;
  }
#pragma unroll
  for (int a = 0; a < NV / kDotBatch + (NV % kDotBatch ? 1 : 0); ++a) {
    if (a * kDotBatch >= nv) break;
    double blk[kDotBatch];
#pragma unroll
    for (int u = 0; u < kDotBatch; ++u) blk[u] = a * kDotBatch + u < NV ? acc[a * kDotBatch + u] : 0.0;
    store_dots<K>(blk, min(kDotBatch, nv - a * kDotBatch), a * kDotBatch, part, pstride);
  }
}

template <int K>
void launch_bmdot(Handle* h, const char* name, unsigned nb, int64_t nk, int nv, const double* V,
                  int64_t ldv, const double* w, double* part, int pstride) {
  if (nv > kFuseMax || !offset_addressable(nk, nb)) {
    LAUNCH(h, name, k_bmdot_part<K>, nb, kT, 0, nk, nv, V, ldv, w, part, pstride);
    return;
  }
  if (nv == 1) {  // the norms of the outer iteration
    LAUNCH(h, name, (k_bmdot<K, 1>), nb, kT, 0, nk, nv, V, ldv, w, part, pstride);
    return;
  }
#define FAMS_DOT(NV) \
  LAUNCH(h, name, (k_bmdot<K, NV>), nb, kT, 0, nk, nv, V, ldv, w, part, pstride)
  switch ((nv + 3) / 4) {
    case 1: FAMS_DOT(4); break;
    case 2: FAMS_DOT(8); break;
    case 3: FAMS_DOT(12); break;
    case 4: FAMS_DOT(16); break;
    case 5: FAMS_DOT(20); break;
    case 6: FAMS_DOT(24); break;
    case 7: FAMS_DOT(28); break;
    case 8: FAMS_DOT(32); break;
  }
#undef FAMS_DOT
}

// the second correction and the norm: w <- w - sum_v coef[r, v] V_v, then
// the partial sums of w^2 per right-hand side, two entries per thread; NV as
// in the fused pass above (loads past nv repeat the last vector with zero
// coefficients)
template <int K, int NV>
__global__ void __launch_bounds__(256) FAMS_STREAM_WAVES
k_bmaxpy_norm(int64_t nk, int nv, const double* V, int64_t ldv, const double* coef, int cstride,
              double* w, double* part) {
  __shared__ double cs[K * NV];
  for (int t = threadIdx.x; t < K * NV; t += blockDim.x) {
    const int r = t / NV, v = t % NV;
    cs[t] = v < nv ? coef[static_cast<int64_t>(r) * cstride + v] : 0.0;
  }
  __syncthreads();
  // the thread's pair of right-hand sides (2 e) % K is fixed: the grid
  // stride is a multiple of 256 pairs
  const double* c0 = cs + ((2 * threadIdx.x) % K) * NV;
  const double* c1 = c0 + NV;
  const char* Vb = reinterpret_cast<const char*>(V);
  char* wb = reinterpret_cast<char*>(w);
  const int64_t ld8 = ldv * 8;
  double a0 = 0.0, a1 = 0.0;
  const uint32_t end = static_cast<uint32_t>((nk / 2) * 16);
  const uint32_t step = gridDim.x * blockDim.x * 16u;
  for (uint32_t off0 = (blockIdx.x * blockDim.x + threadIdx.x) * 16u; off0 < end; off0 += step) {
    const uint32_t off = opaque(off0);
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double2 x = load_at<double2>(Vb + ld8 * min(v, nv - 1), off);
      s0 += c0[v] * x.x;
      s1 += c1[v] * x.y;
    }
    double2 we = load_at<double2>(wb, off);
    we.x -= s0;
    we.y -= s1;
    *reinterpret_cast<double2*>(wb + off) = we;
    a0 += we.x * we.x;
    a1 += we.y * we.y;
  }
  store_pair<K>(a0, a1, 0, part, 1);
}

// the same for any nv and size (restart lengths above kFuseMax, block
// vectors of 4 GiB or more): coefficients read from global memory inside
// the loop over the basis
template <int K>
__global__ void __launch_bounds__(256)
k_bmaxpy_norm_any(int64_t nk, int nv, const double* V, int64_t ldv, const double* coef,
                  int cstride, double* w, double* part) {
  const int64_t n2 = nk / 2;
  double2* w2 = reinterpret_cast<double2*>(w);
  const double* c0 = coef + static_cast<int64_t>((2 * threadIdx.x) % K) * cstride;
  const double* c1 = c0 + cstride;
  double a0 = 0.0, a1 = 0.0;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < n2;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double s0 = 0.0, s1 = 0.0;
    for (int v = 0; v < nv; ++v) {
      const double2 x = reinterpret_cast<const double2*>(V + static_cast<int64_t>(v) * ldv)[e];
      s0 += c0[v] * x.x;
      s1 += c1[v] * x.y;
    }
    double2 we = w2[e];
    we.x -= s0;
    we.y -= s1;
    w2[e] = we;
    a0 += we.x * we.x;
    a1 += we.y * we.y;
  }
  store_pair<K>(a0, a1, 0, part, 1);
}

template <int K>
void launch_bmaxpy_norm(Handle* h, unsigned nb, int64_t nk, int nv, const double* V, int64_t ldv,
                        const double* coef, int cstride, double* w, double* part) {
  if (nv > kFuseMax || !offset_addressable(nk, nb)) {
    LAUNCH(h, "bmaxpy_norm", k_bmaxpy_norm_any<K>, nb, kT, 0, nk, nv, V, ldv, coef, cstride, w,
           part);
    return;
  }
#define FAMS_NORM(NV)                                                                          \
  LAUNCH(h, "bmaxpy_norm", (k_bmaxpy_norm<K, NV>), nb, kT, 0, nk, nv, V, ldv, coef, cstride, w, \
         part)
  switch ((nv + 3) / 4) {
    case 1: FAMS_NORM(4); break;
    case 2: FAMS_NORM(8); break;
    case 3: FAMS_NORM(12); break;
    case 4: FAMS_NORM(16); break;
    case 5: FAMS_NORM(20); break;
    case 6: FAMS_NORM(24); break;
    case 7: FAMS_NORM(28); break;
    case 8: FAMS_NORM(32); break;
  }
#undef FAMS_NORM
}

// out[r * ostride + v] = sum over blocks of the partials of (v, r): one
// workgroup per (v, r), strided partial sums then a fixed tree
__global__ void __launch_bounds__(256)
k_breduce(int nblk, int K, const double* part, int pstride, double* out, int ostride) {
  const int v = blockIdx.x, r = blockIdx.y;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x)
    s += part[(static_cast<int64_t>(b) * pstride + v) * K + r];
  __shared__ double t[4];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  __syncthreads();
  if (threadIdx.x % 64 == 0) t[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[static_cast<int64_t>(r) * ostride + v] = ((t[0] + t[1]) + t[2]) + t[3];
}

// w[i, r] += sign * sum_{v < nv} coef[r * cstride + v] V_v[i, r]
template <int K>
__global__ void k_bmaxpy(int64_t nk, int nv, const double* V, int64_t ldv, const double* coef,
                         int cstride, double sign, double* w) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nk) return;
  const int r = static_cast<int>(e % K);
  const double* c = coef + static_cast<int64_t>(r) * cstride;
  double s = 0.0;
  for (int v = 0; v < nv; ++v) s += c[v] * V[v * ldv + e];
  w[e] += sign * s;
}

// y[i, r] = x[i, r] / d[r * dstride] for the right-hand sides in `mask`,
// 0 for the others
template <int K>
__global__ void k_bscale(int64_t nk, const double* x, const double* d, int dstride, unsigned mask,
                         double* y) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nk) return;
  const int r = static_cast<int>(e % K);
  y[e] = (mask >> r & 1u) ? x[e] / d[static_cast<int64_t>(r) * dstride] : 0.0;
}

// p[i, r] += z[i, r] for the right-hand sides in `mask`
template <int K>
__global__ void k_baxpy_mask(int64_t nk, unsigned mask, const double* z, double* p) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nk) return;
  if (mask >> (e % K) & 1u) p[e] += z[e];
}

__global__ void k_bsqrt(int K, double* d, int stride) {
  const int r = threadIdx.x;
  if (r < K) d[static_cast<int64_t>(r) * stride] = sqrt(d[static_cast<int64_t>(r) * stride]);
}

// per right-hand side GMRES state in one array: S = base + r * stride
struct BState {
  int m, stride;
  int H, cs, sn, g, y, hcol, out, beta;  // offsets inside one right-hand side's record
  int dots, hp, c2, un;                   // the two-pass Gram-Schmidt (see block_gmres)
  static BState make(int m) {
    BState s{};
    s.m = m;
    int o = 0;
    s.H = o; o += (m + 1) * m;
    s.cs = o; o += m;
    s.sn = o; o += m;
    s.g = o; o += m + 1;
    s.y = o; o += m;
    s.hcol = o; o += m + 2;
    s.out = o; o += 2;
    s.beta = o; o += 2;
    s.dots = o; o += 2 * m + 2;
    s.hp = o; o += m + 1;
    s.c2 = o; o += 2 * m + 3;
    s.un = o; o += 2;
    s.stride = o;
    return s;
  }
};

__global__ void k_bgmres_init(int K, BState s, double* base) {
  const int r = threadIdx.x;
  if (r >= K) return;
  double* S = base + static_cast<int64_t>(r) * s.stride;
  for (int k = 0; k <= s.m; ++k) S[s.g + k] = 0.0;
  S[s.g] = S[s.beta];
}

// hcol += y (the second Gram-Schmidt pass), v < nv
__global__ void k_bvadd(int K, int nv, BState s, double* base) {
  const int r = blockIdx.x, v = threadIdx.x;
  if (r < K && v < nv) {
    double* S = base + static_cast<int64_t>(r) * s.stride;
    S[s.hcol + v] += S[s.y + v];
  }
}

// Hessenberg column j, the previous rotations, the new rotation and the
// residual estimate, for every right-hand side in `mask`
__global__ void k_bgivens(int K, BState s, double* base, int j, unsigned mask) {
  const int r = threadIdx.x;
  if (r >= K || !(mask >> r & 1u)) return;
  double* S = base + static_cast<int64_t>(r) * s.stride;
  const int m = s.m;
  double* col = S + s.H + static_cast<int64_t>(j) * (m + 1);
  const double* hcol = S + s.hcol;
  double* cs = S + s.cs;
  double* sn = S + s.sn;
  double* g = S + s.g;
  for (int i = 0; i <= j + 1; ++i) col[i] = hcol[i];
  for (int i = 0; i < j; ++i) {
    const double t = cs[i] * col[i] + sn[i] * col[i + 1];
    col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
    col[i] = t;
  }
  const double den = hypot(col[j], col[j + 1]);
  const double c = den == 0.0 ? 1.0 : col[j] / den;
  const double sg = den == 0.0 ? 0.0 : col[j + 1] / den;
  cs[j] = c;
  sn[j] = sg;
  col[j] = c * col[j] + sg * col[j + 1];
  col[j + 1] = 0.0;
  g[j + 1] = -sg * g[j];
  g[j] = c * g[j];
  S[s.out] = fabs(g[j + 1]);
  S[s.out + 1] = hcol[j + 1];
}

struct KK {
  int v[32];
};

// y = H(0:k, 0:k)^{-1} g(0:k) with each right-hand side's own k; y beyond k
// is zero so that one update over max k columns serves all
__global__ void k_bbacksolve(int K, BState s, double* base, KK kk) {
  const int r = threadIdx.x;
  if (r >= K) return;
  double* S = base + static_cast<int64_t>(r) * s.stride;
  const int m = s.m, k = kk.v[r];
  double* y = S + s.y;
  for (int i = k; i < m; ++i) y[i] = 0.0;
  for (int i = k - 1; i >= 0; --i) {
    double t = S[s.g + i];
    for (int c = i + 1; c < k; ++c) t -= S[s.H + static_cast<int64_t>(c) * (m + 1) + i] * y[c];
    y[i] = t / S[s.H + static_cast<int64_t>(i) * (m + 1) + i];
  }
}

// ---- Gram-Schmidt with the second pass delayed by one step ------------------------
// Each Arnoldi step of block_gmres (two-pass form) reads the basis twice
// instead of three times.  At step j the candidate u_j (V slot j) has been
// orthogonalised once against q_0..q_{j-1} but neither re-orthogonalised nor
// normalised, and w = A M u_j.  Pass one takes, in one sweep over q_0..q_{j-1},
// u_j and w, the dots a = Q^T u_j, b = Q^T w, u_j.u_j and u_j.w.  Then
// q_j = (u_j - Q a) / nu with nu^2 = u_j.u_j - |a|^2 (q_j is orthogonal to Q
// after the second pass, so Pythagoras gives its norm), Hessenberg column
// j - 1 is finished as h' + a with sub-diagonal nu (h' its first-pass
// coefficients), and w's first-pass coefficients against [Q, q_j] are b and
// (u_j.w - a.b) / nu.  Pass two writes q_j into slot j and the next candidate
// u_{j+1} = w - Q b - h_j q_j into slot j + 1, summing |u_{j+1}|^2 for the
// stopping test of column j (taken with the first-pass coefficients; the
// column is finished at step j + 1, or as it stands when its right-hand side
// stops or the cycle ends).  z_j = M u_j is a valid flexible-GMRES direction
// for any u_j, so A Z = V H holds with the finished columns.

// pass one: part[(blk * pstride + i) * K + r] for i < nq: q_i.u, nq + i:
// q_i.w, 2 nq: u.u, 2 nq + 1: u.w (NV >= nq, a multiple of 4, or 0 for nq = 0)
template <int K, int NV>
__global__ void __launch_bounds__(256) FAMS_STREAM_WAVES
k_dcgs_dots(int64_t nk, int nq, const double* V, int64_t ldv, const double* u, const double* w,
            double* part, int pstride) {
  const char* Vb = reinterpret_cast<const char*>(V);
  const char* ub = reinterpret_cast<const char*>(u);
  const char* wb = reinterpret_cast<const char*>(w);
  const int64_t ld8 = ldv * 8;
  double da[NV > 0 ? NV : 1], db[NV > 0 ? NV : 1];
  double duu = 0.0, duw = 0.0;
#pragma unroll
  for (int v = 0; v < (NV > 0 ? NV : 1); ++v) da[v] = db[v] = 0.0;
  const uint32_t end = static_cast<uint32_t>(nk * 8);
  const uint32_t step = gridDim.x * blockDim.x * 8u;
  for (uint32_t off0 = (blockIdx.x * blockDim.x + threadIdx.x) * 8u; off0 < end; off0 += step) {
    const uint32_t off = opaque(off0);
    const double ue = load_at<double>(ub, off);
    const double we = load_at<double>(wb, off);
    if constexpr (NV > 0) {
      double q[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) q[v] = load_at<double>(Vb + ld8 * min(v, nq - 1), off);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        da[v] += q[v] * ue;
        db[v] += q[v] * we;
      }
    }
    duu += ue * ue;
    duw += ue * we;
  }
  // logical order: a (nq), b (nq), u.u, u.w; batches with constant indices
  // so that the sums stay in registers
  constexpr int NB = NV > 0 ? (NV + kDotBatch - 1) / kDotBatch : 0;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      if (a * kDotBatch >= nq) break;
      double blk[kDotBatch];
#pragma unroll
      for (int u = 0; u < kDotBatch; ++u) {
        const int v = a * kDotBatch + u;
        blk[u] = v < NV ? (half ? db[v < NV ? v : 0] : da[v < NV ? v : 0]) : 0.0;
      }
      store_dots<K>(blk, min(kDotBatch, nq - a * kDotBatch), half * nq + a * kDotBatch, part,
                    pstride);
    }
  }
  double tail[kDotBatch] = {duu, duw};
  store_dots<K>(tail, 2, 2 * nq, part, pstride);
}

// pass two, two entries per thread: q_j = (u - sum_i a_i q_i) inv_nu into
// slot nq, u_next = wm w - sum_i b_i q_i - h_j q_j into slot nq + 1, and the
// partial sums of u_next^2.  c2 per right-hand side: a (nq), b (nq), inv_nu,
// h_j, wm (all zero for a right-hand side that has stopped).
template <int K, int NV>
__global__ void __launch_bounds__(256) FAMS_STREAM_WAVES
k_dcgs_update(int64_t nk, int nq, double* V, int64_t ldv, const double* coef, int cstride,
              const double* w, double* part) {
  constexpr int NC = 2 * (NV > 0 ? NV : 0) + 3;
  __shared__ double cs[K * NC];
  for (int t = threadIdx.x; t < K * NC; t += blockDim.x) {
    const int r = t / NC, v = t % NC;
    double c = 0.0;
    if (v < NV) c = v < nq ? coef[static_cast<int64_t>(r) * cstride + v] : 0.0;
    else if (v < 2 * NV) c = v - NV < nq ? coef[static_cast<int64_t>(r) * cstride + nq + v - NV] : 0.0;
    else c = coef[static_cast<int64_t>(r) * cstride + 2 * nq + (v - 2 * NV)];
    cs[t] = c;
  }
  __syncthreads();
  const int r0 = (2 * threadIdx.x) % K;
  const double* c0 = cs + r0 * NC;
  const double* c1 = c0 + NC;
  char* Vb = reinterpret_cast<char*>(V);
  const char* wb = reinterpret_cast<const char*>(w);
  const int64_t ld8 = ldv * 8;
  char* ub = Vb + ld8 * nq;
  char* nb_ = Vb + ld8 * (nq + 1);
  double a0 = 0.0, a1 = 0.0;
  const uint32_t end = static_cast<uint32_t>((nk / 2) * 16);
  const uint32_t step = gridDim.x * blockDim.x * 16u;
  for (uint32_t off0 = (blockIdx.x * blockDim.x + threadIdx.x) * 16u; off0 < end; off0 += step) {
    const uint32_t off = opaque(off0);
    const double2 ue = load_at<double2>(ub, off);
    const double2 we = load_at<double2>(wb, off);
    double sa0 = 0.0, sa1 = 0.0, sb0 = 0.0, sb1 = 0.0;
    if constexpr (NV > 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double2 x = load_at<double2>(Vb + ld8 * min(v, nq - 1), off);
        sa0 += c0[v] * x.x;
        sa1 += c1[v] * x.y;
        sb0 += c0[NV + v] * x.x;
        sb1 += c1[NV + v] * x.y;
      }
    }
    double2 qv, un;
    qv.x = (ue.x - sa0) * c0[2 * NV];
    qv.y = (ue.y - sa1) * c1[2 * NV];
    un.x = c0[2 * NV + 2] * we.x - sb0 - c0[2 * NV + 1] * qv.x;
    un.y = c1[2 * NV + 2] * we.y - sb1 - c1[2 * NV + 1] * qv.y;
    *reinterpret_cast<double2*>(ub + off) = qv;
    *reinterpret_cast<double2*>(nb_ + off) = un;
    a0 += un.x * un.x;
    a1 += un.y * un.y;
  }
  store_pair<K>(a0, a1, 0, part, 1);
}

template <int K>
void launch_dcgs(Handle* h, bool second, unsigned nb, int64_t nk, int nq, double* V, int64_t ldv,
                 const double* w, const double* coef, int cstride, double* part, int pstride) {
#define FAMS_DCGS(NV)                                                                          \
  do {                                                                                         \
    if (second)                                                                                \
      LAUNCH(h, "bgs_update", (k_dcgs_update<K, NV>), nb, kT, 0, nk, nq, V, ldv, coef,         \
             cstride, w, part);                                                                \
    else                                                                                       \
      LAUNCH(h, "bgs_dots", (k_dcgs_dots<K, NV>), nb, kT, 0, nk, nq, V, ldv,                   \
             static_cast<const double*>(V + static_cast<int64_t>(nq) * ldv), w, part, pstride); \
  } while (0)
  switch ((nq + 3) / 4) {
    case 0: FAMS_DCGS(0); break;
    case 1: FAMS_DCGS(4); break;
    case 2: FAMS_DCGS(8); break;
    case 3: FAMS_DCGS(12); break;
    case 4: FAMS_DCGS(16); break;
    case 5: FAMS_DCGS(20); break;
    case 6: FAMS_DCGS(24); break;
    case 7: FAMS_DCGS(28); break;
    case 8: FAMS_DCGS(32); break;
    default: FAMS_REQUIRE(false, FAMS_ERR_CAPACITY, "two-pass Gram-Schmidt: too many vectors");
  }
#undef FAMS_DCGS
}

// per right-hand side in `mask` (one thread each): finish Hessenberg column
// j - 1 from its first-pass coefficients and the dots of pass one (rotations
// 0..j-2 applied, rotation j-1 formed, g updated), keep w's first-pass
// coefficients for column j, and set pass two's coefficients; right-hand
// sides outside the mask get zero coefficients.  A candidate without a part
// orthogonal to Q (nu^2 <= 0) gets a zero q_j and is flagged (out[1] = 0).
__global__ void k_dcgs_coef(int K, BState s, double* base, int j, unsigned mask) {
  const int r = threadIdx.x;
  if (r >= K) return;
  double* S = base + static_cast<int64_t>(r) * s.stride;
  double* c2 = S + s.c2;
  if (!(mask >> r & 1u)) {
    for (int i = 0; i < 2 * j + 3; ++i) c2[i] = 0.0;
    return;
  }
  const int m = s.m;
  const double* a = S + s.dots;
  const double* b = a + j;
  const double uu = a[2 * j], uw = a[2 * j + 1];
  double na2 = 0.0, ab = 0.0;
  for (int i = 0; i < j; ++i) {
    na2 += a[i] * a[i];
    ab += a[i] * b[i];
  }
  const double nu2 = uu - na2;
  const double nu = nu2 > 0.0 ? sqrt(nu2) : 0.0;
  const double inv = nu > 0.0 ? 1.0 / nu : 0.0;
  S[s.un + 1] = nu > 0.0 ? 1.0 : 0.0;
  if (j >= 1) {
    double* col = S + s.H + static_cast<int64_t>(j - 1) * (m + 1);
    double* cs = S + s.cs;
    double* sn = S + s.sn;
    double* g = S + s.g;
    const double* hp = S + s.hp;
    for (int i = 0; i < j; ++i) col[i] = hp[i] + a[i];
    col[j] = nu;
    for (int i = 0; i < j - 1; ++i) {
      const double t = cs[i] * col[i] + sn[i] * col[i + 1];
      col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
      col[i] = t;
    }
    const double den = hypot(col[j - 1], col[j]);
    const double c = den == 0.0 ? 1.0 : col[j - 1] / den;
    const double sg = den == 0.0 ? 0.0 : col[j] / den;
    cs[j - 1] = c;
    sn[j - 1] = sg;
    col[j - 1] = c * col[j - 1] + sg * col[j];
    col[j] = 0.0;
    g[j] = -sg * g[j - 1];
    g[j - 1] = c * g[j - 1];
  }
  double* hp = S + s.hp;
  for (int i = 0; i < j; ++i) hp[i] = b[i];
  const double hj = (uw - ab) * inv;
  hp[j] = hj;
  for (int i = 0; i < j; ++i) {
    c2[i] = a[i];
    c2[j + i] = b[i];
  }
  c2[2 * j] = inv;
  c2[2 * j + 1] = hj;
  c2[2 * j + 2] = 1.0;
}

// the stopping test of column j from its first-pass coefficients: hcol = [h',
// |u_{j+1}|] (what k_bgivens commits when the column ends here), out[0] = the
// residual estimate after the rotations, out[1] = |u_{j+1}| (0 if flagged)
__global__ void k_dcgs_estimate(int K, BState s, double* base, int j, unsigned mask) {
  const int r = threadIdx.x;
  if (r >= K || !(mask >> r & 1u)) return;
  double* S = base + static_cast<int64_t>(r) * s.stride;
  const double t = sqrt(fmax(S[s.un], 0.0));
  double* hcol = S + s.hcol;
  for (int i = 0; i <= j; ++i) hcol[i] = S[s.hp + i];
  hcol[j + 1] = t;
  // entry j after rotations 0..j-1 (rotation i turns rows i and i + 1; the
  // running value is row i + 1's after it)
  double x = hcol[0];
  for (int i = 0; i < j; ++i) x = -S[s.sn + i] * x + S[s.cs + i] * hcol[i + 1];
  const double y = t;
  const double den = hypot(x, y);
  const double sg = den == 0.0 ? 0.0 : y / den;
  S[s.out] = fabs(sg * S[s.g + j]);
  S[s.out + 1] = S[s.un + 1] > 0.0 ? t : 0.0;
}

// ---- the lock-step iteration -----------------------------------------------------
struct BWork {
  int K, m;
  int64_t nk;
  double *q, *p, *r, *w, *d1, *z, *rh, *x, *y, *xb, *V, *Z;
  float *r32, *d1_32, *rh32, *x32, *y32, *xb32;
  double *rc, *xc, *cpart;
  int cw, nch;
  double* part;
  int nb;
  double* small;
  BState st;
};

size_t block_vectors(int m) { return static_cast<size_t>(10 + 2 * m + 1); }

int coarse_chunk_width(int nc) { return 64 * std::max(1, (nc + 64 * 32 - 1) / (64 * 32)); }

BWork block_work(Handle* h, int K, int m) {
  BWork k{};
  const int64_t n = h->n;
  k.K = K;
  k.m = m;
  k.nk = n * K;
  double* b = h->bwk.get();
  double** seq[] = {&k.q, &k.p, &k.r, &k.w, &k.d1, &k.z, &k.rh, &k.x, &k.y, &k.xb};
  for (double** s : seq) {
    *s = b;
    b += k.nk;
  }
  k.V = b;
  k.Z = k.V + static_cast<int64_t>(m + 1) * k.nk;
  if (h->precision == FAMS_PREC_MIXED) {
    float* f = h->bwk32.get();
    float** s32[] = {&k.r32, &k.d1_32, &k.rh32, &k.x32, &k.y32, &k.xb32};
    for (float** s : s32) {
      *s = f;
      f += k.nk;
    }
  }
  k.cw = coarse_chunk_width(h->nc);
  k.nch = (h->nc + k.cw - 1) / k.cw;
  k.rc = h->bpart.get();
  k.xc = k.rc + static_cast<int64_t>(h->nc) * K;
  k.cpart = k.xc + static_cast<int64_t>(h->nc) * K;
  k.part = h->bred.get();
  k.nb = static_cast<int>(std::min<int64_t>(kRedBlocks, blocks_for(k.nk, kT)));
  k.st = BState::make(m);
  k.small = h->bsmall.get();
  return k;
}

size_t block_bytes(Handle* h, int K, int m) {
  const size_t nk = static_cast<size_t>(h->n) * K;
  size_t b = block_vectors(m) * nk * sizeof(double);
  if (h->precision == FAMS_PREC_MIXED) b += 6 * nk * sizeof(float);
  const int cw = coarse_chunk_width(h->nc);
  const size_t nch = (h->nc + cw - 1) / cw;
  b += (2 + nch) * static_cast<size_t>(h->nc) * K * sizeof(double);
  return b;
}

// forward column offsets (j - i, j in the first nm rows) of up to 8 entries
// of each of S rows spread evenly over the first nm rows; 0 fills the rest
constexpr int kTileSample = 4096;
__global__ void k_offset_sample(int nm, const int* rp, const int* ci, int* out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= kTileSample) return;
  const int i = static_cast<int>(static_cast<int64_t>(s) * nm / kTileSample);
  int k = 0;
  for (int p = rp[i]; p < rp[i + 1] && k < 8; ++p) {
    const int j = ci[p];
    if (j > i && j < nm) out[s * 8 + k++] = j - i;
  }
  for (; k < 8; ++k) out[s * 8 + k] = 0;
}

// The grid behind the first nm rows, read off the sample: offset 1 and two
// larger offsets sy < sz, each in at least half of the sampled rows, with
// sz a multiple of sy and nm a multiple of sz (then the slab order is a
// permutation of the nm rows whatever the matrix is).  Anything else, or a
// grid too small to gain, keeps natural order.
RowTiling infer_tiling(Handle* h) {
  RowTiling t;
  const int nm = h->nm;
  if (nm < 4096) return t;
  DBuf<int> d(&h->alloc, kTileSample * 8);
  LAUNCH(h, "btiling", k_offset_sample, blocks_for(kTileSample, 256), 256, 0, nm, h->rp.get(),
         h->ci.get(), d.get());
  std::vector<int> off(kTileSample * 8);
  HIPX(hipMemcpyAsync(off.data(), d.get(), off.size() * sizeof(int), hipMemcpyDeviceToHost,
                      h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  std::map<int, int> hist;
  for (int v : off)
    if (v > 0) ++hist[v];
  int sy = 0, sz = 0, cy = 0, cz = 0;  // the two most frequent offsets above 1
  for (const auto& [v, c] : hist) {
    if (v == 1) continue;
    if (c > cy) {
      sz = sy; cz = cy;
      sy = v; cy = c;
    } else if (c > cz) {
      sz = v; cz = c;
    }
  }
  if (sy > sz) std::swap(sy, sz), std::swap(cy, cz);
  const int half = kTileSample / 2;
  if (hist.count(1) == 0 || hist[1] < half || cy < half || cz < half || sy < 2 || sz % sy != 0 ||
      nm % sz != 0)
    return t;
  t.nm = nm;
  t.sy = sy;
  t.ny = sz / sy;
  t.nz = nm / sz;
  t.yb = std::max(1, std::min(t.ny, 4096 / sy));  // a slab plane of ~4096 rows
  if (t.nz < 2) t = RowTiling{};
  return t;
}

void free_block_workspace(Handle* h) {
  h->bK = 0;
  h->bwk.free();
  h->bwk32.free();
  h->bpart.free();
  h->bred.free();
  h->bsmall.free();
}

// all or nothing: a failed allocation leaves no work space (bK = 0)
void ensure_block_workspace(Handle* h, int K, int m) {
  if (!h->tiling_known) {
    h->tiling = infer_tiling(h);
    h->tiling_known = true;
    h->info.tiled_rows = h->tiling.sy ? h->tiling.nm : 0;
  }
  if (h->bK == K && h->bm >= m && h->bwk.get()) return;
  free_block_workspace(h);
  try {
    const size_t nk = static_cast<size_t>(h->n) * K;
    h->bwk.reset(&h->alloc, block_vectors(m) * nk);
    if (h->precision == FAMS_PREC_MIXED) h->bwk32.reset(&h->alloc, 6 * nk);
    const int cw = coarse_chunk_width(h->nc);
    const size_t nch = (h->nc + cw - 1) / cw;
    h->bpart.reset(&h->alloc, (2 + nch) * static_cast<size_t>(h->nc) * K);
    h->bred.reset(&h->alloc, static_cast<size_t>(kRedBlocks) * (2 * m + 4) * K + 16);
    h->bsmall.reset(&h->alloc, static_cast<size_t>(BState::make(m).stride) * K + 16);
  } catch (...) {
    free_block_workspace(h);
    throw;
  }
  h->bK = K;
  h->bm = m;
}

// the fixed-width form of the CSR matrix (rp, ci, val, val32) with values
// of type TV, built on first use
template <class TV>
const TV* ell_vals(Handle* h, EllMat& e, const int* rp, const int* ci, const double* val,
                   const float* val32) {
  const int n = h->n;
  if (!e.col.get()) {
    e.col.reset(&h->alloc, static_cast<size_t>(n) * kEll);
    e.ovf.reset(&h->alloc, 2 * static_cast<size_t>(n));
    LAUNCH(h, "bell", k_ell_cols, blocks_for(n, 256), 256, 0, n, rp, ci, e.col.get(),
           e.ovf.get());
  }
  if constexpr (std::is_same<TV, double>::value) {
    if (!e.val.get()) {
      e.val.reset(&h->alloc, static_cast<size_t>(n) * kEll);
      LAUNCH(h, "bell", k_ell_vals<double>, blocks_for(n, 256), 256, 0, n, rp, val, e.val.get());
    }
    return e.val.get();
  } else {
    if (!e.val32.get()) {
      e.val32.reset(&h->alloc, static_cast<size_t>(n) * kEll);
      LAUNCH(h, "bell", k_ell_vals<float>, blocks_for(n, 256), 256, 0, n, rp, val32,
             e.val32.get());
    }
    return e.val32.get();
  }
}

// y = b - A x (kResid; "bspmv_resid" inside the stage, "bresid_outer" for the
// FP64 residual of the outer iteration) or y = A x ("bspmv") on block vectors
template <class TV, class TX, class TB, class TY, int K, bool kResid>
void aprod(Handle* h, const TX* x, const TB* b, TY* y, const char* name) {
  const int64_t nk = static_cast<int64_t>(h->n) * K;
  const TV* ev = ell_vals<TV>(h, h->ell, h->rp.get(), h->ci.get(), h->val.get(), h->val32.get());
  const TV* cv;
  if constexpr (std::is_same<TV, double>::value) cv = h->val.get();
  else cv = h->val32.get();
  LAUNCH(h, name, (k_bspmv_ell<TV, TX, TB, TY, K, kResid>), xcd_grid(blocks_for(nk / 2, kT)), kT,
         0, h->n, h->ell.col.get(), ev, h->ell.ovf.get(), h->ci.get(), cv, x, b, y, h->tiling);
}

// y = P x on block vectors (natural row order: the gathered coarse values
// stay in L2 whatever the order)
template <class TV, int K>
void pprod(Handle* h, const double* x, TV* y) {
  const int64_t nk = static_cast<int64_t>(h->n) * K;
  const TV* ev = ell_vals<TV>(h, h->pell, h->p_rp.get(), h->p_ci.get(), h->p_val.get(),
                              h->p_val32.get());
  const TV* cv;
  if constexpr (std::is_same<TV, double>::value) cv = h->p_val.get();
  else cv = h->p_val32.get();
  LAUNCH(h, "bprolong", (k_bspmv_ell<TV, double, TV, TV, K, false>),
         xcd_grid(blocks_for(nk / 2, kT)), kT, 0, h->n, h->pell.col.get(), ev, h->pell.ovf.get(),
         h->p_ci.get(), cv, x, static_cast<const TV*>(nullptr), y, RowTiling{});
}

template <class TV, class TX, class TB, class TY, int K>
void bresid(Handle* h, const TX* x, const TB* b, TY* y, const char* name = "bspmv_resid") {
  aprod<TV, TX, TB, TY, K, true>(h, x, b, y, name);
}

// Table 1 steps 5-7 on K residuals at once (FP64 in and out; T = stage type)
template <class T, int K>
void bstage(Handle* h, const BWork& k, const double* r, double* z) {
  const int n = h->n, nc = h->nc;
  const int64_t nk = k.nk;
  const T *rv, *lu;
  const T* rT;
  T *d1, *rh, *x, *ysc, *xb;
  if constexpr (std::is_same<T, double>::value) {
    rv = h->r_val.get();
    lu = h->ilu.get();
    rT = r;
    d1 = k.d1;
    rh = k.rh;
    x = k.x;
    ysc = k.y;
    xb = k.xb;
  } else {
    rv = h->r_val32.get();
    lu = h->ilu32.get();
    LAUNCH(h, "bcast_d2f", (k_bcast<double, float>), blocks_for(nk, kT), kT, 0, nk, r, k.r32);
    rT = k.r32;
    d1 = k.d1_32;
    rh = k.rh32;
    x = k.x32;
    ysc = k.y32;
    xb = k.xb32;
  }
  LAUNCH(h, "brestrict", (k_brestrict<T, T, K>), nc, 256, 0, nc, h->r_rp.get(), h->r_ci.get(),
         rv, rT, k.rc);
  {
    if constexpr (K % 16 == 0) {
      dim3 grid(blocks_for(nc, 64), k.nch);
      LAUNCH(h, "bcoarse", k_bcoarse_mfma<K>, grid, 256, 0, nc, k.cw, h->Ainv.get(), k.rc,
             k.cpart);
    } else {
      dim3 grid(blocks_for(nc, 256), k.nch);
      LAUNCH(h, "bcoarse", k_bcoarse_part<K>, grid, 256, 0, nc, k.cw, h->Ainv.get(), k.rc,
             k.cpart);
    }
    const int64_t nck = static_cast<int64_t>(nc) * K;
    LAUNCH(h, "bcoarse_red", k_bcoarse_red, blocks_for(nck, kT), kT, 0, nck, k.nch, k.cpart, k.xc);
  }
  pprod<T, K>(h, k.xc, d1);
  if (h->smoother) {
    bresid<T, T, T, T, K>(h, d1, rT, rh);
    if (!h->blk) {  // z = d1 + x written by the upper sweep as each row finishes
      ilu_apply_block<T, K>(h, lu, rh, x, ysc, d1, z);
      return;
    }
    ilu_apply_block<T, K>(h, lu, rh, x, ysc);
    {  // per-medium stage on the residual left by the ILU(0) stage
      Handle* b = h->blk.get();
      const T* blu;
      if constexpr (std::is_same<T, double>::value) blu = b->ilu.get();
      else blu = b->ilu32.get();
      bresid<T, T, T, T, K>(h, x, rh, rh);
      ilu_apply_block<T, K>(b, blu, rh, xb, ysc);
      LAUNCH(h, "badd", (k_badd<T, T, T>), blocks_for(nk, kT), kT, 0, nk, x, xb, x);
    }
    LAUNCH(h, "badd", (k_badd<T, T, double>), blocks_for(nk, kT), kT, 0, nk, d1, x, z);
  } else {
    LAUNCH(h, "bcast", (k_bcast<T, double>), blocks_for(nk, kT), kT, 0, nk, d1, z);
  }
}

template <int K>
void bstage_any(Handle* h, const BWork& k, const double* r, double* z) {
  if (h->precision == FAMS_PREC_MIXED) bstage<float, K>(h, k, r, z);
  else bstage<double, K>(h, k, r, z);
}

// ||x_r|| of every right-hand side into S[r * stride + off]
template <int K>
void bnorms(Handle* h, const BWork& k, const double* x, int off) {
  launch_bmdot<K>(h, "bdot", k.nb, k.nk, 1, x, k.nk, x, k.part, 1);
  LAUNCH(h, "breduce", k_breduce, dim3(1, K), 256, 0, k.nb, K, k.part, 1, k.small + off,
         k.st.stride);
  LAUNCH(h, "bsqrt", k_bsqrt, 1, 64, 0, K, k.small + off, k.st.stride);
}

std::vector<double> read_field(Handle* h, const BWork& k, int off, int cnt) {
  std::vector<double> all(static_cast<size_t>(k.st.stride) * k.K);
  HIPX(hipMemcpyAsync(all.data(), k.small, all.size() * sizeof(double), hipMemcpyDeviceToHost,
                      h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  std::vector<double> v(static_cast<size_t>(k.K) * cnt);
  for (int r = 0; r < k.K; ++r)
    for (int c = 0; c < cnt; ++c) v[r * cnt + c] = all[static_cast<size_t>(r) * k.st.stride + off + c];
  return v;
}

struct RhsState {
  double r0 = 0.0, tol = 0.0, beta = 0.0;
  int it = 0;
  bool done = false;
  fams_status_t st = FAMS_NOT_CONVERGED;
};

// the stopping tests at a restart (or a Table 1 step), from the true residual
void check_rhs(RhsState& s, int max_iter) {
  if (s.done) return;
  if (s.beta <= s.tol) {
    s.st = FAMS_OK;
    s.done = true;
  } else if (!std::isfinite(s.beta) || s.beta > 1e8 * s.r0) {
    s.st = FAMS_DIVERGED;
    s.done = true;
  } else if (s.it >= max_iter) {
    s.done = true;
  }
}

template <int K>
void block_gmres(Handle* h, const BWork& k, int nr, const fams_solve_opts_t* o,
                 std::vector<RhsState>& rs) {
  const int64_t n = h->n, nk = k.nk;
  const int m = std::min(o->restart, k.m);
  const BState& S = k.st;
  // Gram-Schmidt: the two-pass form (second pass of each candidate delayed to
  // the next step) while its fused kernels can take the basis, else CGS2
  // with three passes
  const bool two_pass = m <= kFuseMax && offset_addressable(nk, k.nb);
  bresid<double, double, double, double, K>(h, k.p, k.q, k.r, "bresid_outer");
  bnorms<K>(h, k, k.r, S.beta);
  std::vector<double> b = read_field(h, k, S.beta, 1);
  for (int r = 0; r < K; ++r) {
    rs[r].r0 = rs[r].beta = b[r];
    rs[r].tol = o->rtol * b[r];
    if (r >= nr) {  // padding lanes
      rs[r].done = true;
      rs[r].st = FAMS_OK;
    }
    if (rs[r].r0 == 0.0 && !rs[r].done) {
      rs[r].done = true;
      rs[r].st = FAMS_OK;
    }
  }
  (void)n;
  while (true) {
    unsigned mask = 0;
    for (int r = 0; r < K; ++r) {
      check_rhs(rs[r], o->max_iter);
      if (!rs[r].done) mask |= 1u << r;
    }
    if (!mask) break;
    LAUNCH(h, "bscale", k_bscale<K>, blocks_for(nk, kT), kT, 0, nk, k.r, k.small + S.beta,
           S.stride, mask, k.V);
    LAUNCH(h, "bgmres_init", k_bgmres_init, 1, 64, 0, K, S, k.small);
    KK kk{};
    unsigned cyc = mask;
    int jmax = 0;
    if (two_pass) {
      for (int j = 0; j < m && cyc; ++j) {
        double* uj = k.V + j * nk;
        double* zj = k.Z + j * nk;
        bstage_any<K>(h, k, uj, zj);
        aprod<double, double, double, double, K, false>(h, zj, static_cast<const double*>(nullptr),
                                                        k.w, "bspmv");
        launch_dcgs<K>(h, false, k.nb, nk, j, k.V, nk, k.w, nullptr, 0, k.part, 2 * m + 2);
        LAUNCH(h, "breduce", k_breduce, dim3(2 * j + 2, K), 256, 0, k.nb, K, k.part, 2 * m + 2,
               k.small + S.dots, S.stride);
        LAUNCH(h, "bgs_coef", k_dcgs_coef, 1, 64, 0, K, S, k.small, j, cyc);
        launch_dcgs<K>(h, true, k.nb, nk, j, k.V, nk, k.w, k.small + S.c2, S.stride, k.part, 1);
        LAUNCH(h, "breduce", k_breduce, dim3(1, K), 256, 0, k.nb, K, k.part, 1, k.small + S.un,
               S.stride);
        LAUNCH(h, "bgs_estimate", k_dcgs_estimate, 1, 64, 0, K, S, k.small, j, cyc);
        std::vector<double> est = read_field(h, k, S.out, 2);
        unsigned next = 0;
        for (int r = 0; r < K; ++r) {
          if (!(cyc >> r & 1u)) continue;
          ++rs[r].it;
          kk.v[r] = j + 1;
          const double e = est[2 * r], hn = est[2 * r + 1];
          if (!(e <= rs[r].tol || rs[r].it >= o->max_iter || !(hn > 0.0) || !std::isfinite(e)))
            next |= 1u << r;
        }
        jmax = j + 1;
        // columns that end here (their right-hand side stops, or the cycle
        // ends) are committed as they stand
        const unsigned commit = j + 1 == m ? cyc : (cyc & ~next);
        if (commit) LAUNCH(h, "bgivens", k_bgivens, 1, 64, 0, K, S, k.small, j, commit);
        cyc = next;
      }
    }
    for (int j = 0; j < m && cyc && !two_pass; ++j) {
      double* vj = k.V + j * nk;
      double* zj = k.Z + j * nk;
      bstage_any<K>(h, k, vj, zj);
      aprod<double, double, double, double, K, false>(h, zj, static_cast<const double*>(nullptr),
                                                      k.w, "bspmv");
      // CGS2 against V_0..V_j, per right-hand side: h = V^T w; w -= V h and
      // c = V^T w in one pass; w -= V c and ||w|| in one pass; h += c
      launch_bmdot<K>(h, "bmdot", k.nb, nk, j + 1, k.V, nk, k.w, k.part, m + 2);
      LAUNCH(h, "breduce", k_breduce, dim3(j + 1, K), 256, 0, k.nb, K, k.part, m + 2,
             k.small + S.hcol, S.stride);
      if (j + 1 <= kFuseMax && offset_addressable(nk, k.nb)) {
        launch_bmaxpy_mdot<K>(h, k.nb, nk, j + 1, k.V, nk, k.small + S.hcol, S.stride, k.w,
                              k.part, m + 2);
      } else {  // more basis vectors than the fused pass holds sums for
        LAUNCH(h, "bmaxpy", k_bmaxpy<K>, blocks_for(nk, kT), kT, 0, nk, j + 1, k.V, nk,
               k.small + S.hcol, S.stride, -1.0, k.w);
        LAUNCH(h, "bmdot", k_bmdot_part<K>, k.nb, kT, 0, nk, j + 1, k.V, nk, k.w, k.part, m + 2);
      }
      LAUNCH(h, "breduce", k_breduce, dim3(j + 1, K), 256, 0, k.nb, K, k.part, m + 2,
             k.small + S.y, S.stride);
      launch_bmaxpy_norm<K>(h, k.nb, nk, j + 1, k.V, nk, k.small + S.y, S.stride, k.w, k.part);
      LAUNCH(h, "breduce", k_breduce, dim3(1, K), 256, 0, k.nb, K, k.part, 1,
             k.small + S.hcol + j + 1, S.stride);
      LAUNCH(h, "bsqrt", k_bsqrt, 1, 64, 0, K, k.small + S.hcol + j + 1, S.stride);
      LAUNCH(h, "bvadd", k_bvadd, K, 64, 0, K, j + 1, S, k.small);
      LAUNCH(h, "bgivens", k_bgivens, 1, 64, 0, K, S, k.small, j, cyc);
      std::vector<double> est = read_field(h, k, S.out, 2);
      unsigned next = 0;
      for (int r = 0; r < K; ++r) {
        if (!(cyc >> r & 1u)) continue;
        ++rs[r].it;
        kk.v[r] = j + 1;
        const double e = est[2 * r], hn = est[2 * r + 1];
        if (!(e <= rs[r].tol || rs[r].it >= o->max_iter || !(hn > 0.0) || !std::isfinite(e)))
          next |= 1u << r;
      }
      jmax = j + 1;
      cyc = next;
      if (cyc)
        LAUNCH(h, "bscale", k_bscale<K>, blocks_for(nk, kT), kT, 0, nk, k.w, k.small + S.hcol + j + 1,
               S.stride, cyc, k.V + (j + 1) * nk);
    }
    LAUNCH(h, "bbacksolve", k_bbacksolve, 1, 64, 0, K, S, k.small, kk);
    LAUNCH(h, "bmaxpy", k_bmaxpy<K>, blocks_for(nk, kT), kT, 0, nk, jmax, k.Z, nk, k.small + S.y,
           S.stride, 1.0, k.p);
    bresid<double, double, double, double, K>(h, k.p, k.q, k.r, "bresid_outer");
    bnorms<K>(h, k, k.r, S.beta);
    b = read_field(h, k, S.beta, 1);
    for (int r = 0; r < K; ++r)
      if (!rs[r].done) rs[r].beta = b[r];
  }
}

template <int K>
void block_richardson(Handle* h, const BWork& k, int nr, const fams_solve_opts_t* o,
                      std::vector<RhsState>& rs) {
  const int64_t nk = k.nk;
  const BState& S = k.st;
  bresid<double, double, double, double, K>(h, k.p, k.q, k.r, "bresid_outer");
  bnorms<K>(h, k, k.r, S.beta);
  std::vector<double> b = read_field(h, k, S.beta, 1);
  for (int r = 0; r < K; ++r) {
    rs[r].r0 = rs[r].beta = b[r];
    rs[r].tol = o->rtol * b[r];
    if (r >= nr || b[r] == 0.0) {
      rs[r].done = true;
      rs[r].st = FAMS_OK;
    }
  }
  while (true) {
    unsigned mask = 0;
    for (int r = 0; r < K; ++r) {
      check_rhs(rs[r], o->max_iter);
      if (!rs[r].done) mask |= 1u << r;
    }
    if (!mask) break;
    bstage_any<K>(h, k, k.r, k.z);
    LAUNCH(h, "baxpy", k_baxpy_mask<K>, blocks_for(nk, kT), kT, 0, nk, mask, k.z, k.p);
    bresid<double, double, double, double, K>(h, k.p, k.q, k.r, "bresid_outer");
    bnorms<K>(h, k, k.r, S.beta);
    b = read_field(h, k, S.beta, 1);
    for (int r = 0; r < K; ++r)
      if (mask >> r & 1u) {
        ++rs[r].it;
        rs[r].beta = b[r];
      }
  }
}

template <int K>
void solve_group(Handle* h, const double* q, double* p, int nr, const fams_solve_opts_t* o,
                 fams_info_t* info) {
  const int m = o->outer == FAMS_GMRES ? o->restart : 1;
  ensure_block_workspace(h, K, m);
  BWork k = block_work(h, K, m);
  const int n = h->n;
  const int64_t nk = k.nk;
  for (Handle* g : {h, h->blk.get()})
    if (g && g->sweep_err.get()) HIPX(hipMemsetAsync(g->sweep_err, 0, 2 * sizeof(int), h->stream));
  auto t0 = std::chrono::steady_clock::now();
  LAUNCH(h, "bpack", k_pack<K>, blocks_for(n, kPackRows), kT, 0, n, nr, q, k.q);
  if (o->use_initial_guess)
    LAUNCH(h, "bpack", k_pack<K>, blocks_for(n, kPackRows), kT, 0, n, nr, static_cast<const double*>(p),
           k.p);
  else
    HIPX(hipMemsetAsync(k.p, 0, nk * sizeof(double), h->stream));
  std::vector<RhsState> rs(K);
  if (o->outer == FAMS_GMRES) block_gmres<K>(h, k, nr, o, rs);
  else block_richardson<K>(h, k, nr, o, rs);
  LAUNCH(h, "bunpack", k_unpack<K>, blocks_for(n, kPackRows), kT, 0, n, nr, k.p, p);
  HIPX(hipStreamSynchronize(h->stream));
  int e = 0;
  for (Handle* g : {h, h->blk.get()}) {
    if (!g || !g->sweep_err.get()) continue;
    int eg[2] = {};
    HIPX(hipMemcpyAsync(eg, g->sweep_err.get(), sizeof(eg), hipMemcpyDeviceToHost, h->stream));
    HIPX(hipStreamSynchronize(h->stream));
    e |= eg[0];
    h->info.long_waits += eg[1];
  }
  FAMS_REQUIRE(e == 0, FAMS_ERR_DEVICE, "ILU(0) sweep: a dependency wait exceeded its bound");
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (int r = 0; r < nr; ++r) {
    info[r].status = rs[r].st;
    info[r].iterations = rs[r].it;
    info[r].rel_residual = rs[r].r0 > 0 ? rs[r].beta / rs[r].r0 : 0.0;
    info[r].ms = ms;
  }
}

}  // namespace

fams_status_t solve_block(Handle* h, const double* q, double* p, int nrhs,
                          const fams_solve_opts_t* o, fams_info_t* info) {
  const int m = o->outer == FAMS_GMRES ? o->restart : 1;
  // the widest group (up to 32 right-hand sides, no wider than nrhs needs)
  // whose work space fits in the device memory
  int K = 32;
  while (K > 2 && K / 2 >= nrhs) K /= 2;
  size_t free_b = 0, total_b = 0;
  HIPX(hipMemGetInfo(&free_b, &total_b));
  if (!h->alloc.has_hook) {
    // the free device memory, with a margin for the caller
    const size_t held = h->bwk.get() ? block_bytes(h, h->bK, h->bm) : 0;
    while (K > 2 && block_bytes(h, K, m) > (free_b + held) / 10 * 9) K /= 2;
    FAMS_REQUIRE(block_bytes(h, K, m) <= free_b + held, FAMS_ERR_OOM,
                 "no room for the lock-step work space of two right-hand sides");
  } else {
    // an allocation hook may hold memory that the device does not count as
    // free (a caching allocator): ask the hook for the widest work space and
    // halve the group while it refuses
    while (K > 2 && block_bytes(h, K, m) > total_b) K /= 2;
    for (;;) {
      try {
        ensure_block_workspace(h, K, m);
        break;
      } catch (const Error& e) {
        if (e.status != FAMS_ERR_OOM || K == 2) throw;
        K /= 2;
      }
    }
  }
  const int64_t n = h->n;
  fams_status_t worst = FAMS_OK;
  for (int r0 = 0; r0 < nrhs; r0 += K) {
    const int nr = std::min(K, nrhs - r0);
    fams_info_t* inf = info + r0;
    const double* qg = q + r0 * n;
    double* pg = p + r0 * n;
    switch (K) {
      case 2: solve_group<2>(h, qg, pg, nr, o, inf); break;
      case 4: solve_group<4>(h, qg, pg, nr, o, inf); break;
      case 8: solve_group<8>(h, qg, pg, nr, o, inf); break;
      case 16: solve_group<16>(h, qg, pg, nr, o, inf); break;
      default: solve_group<32>(h, qg, pg, nr, o, inf); break;
    }
    for (int r = 0; r < nr; ++r)
      if (inf[r].status > worst) worst = static_cast<fams_status_t>(inf[r].status);
  }
  return worst;
}

}  // namespace fams
