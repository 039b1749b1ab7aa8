// Setup, part 2, and the coarse solve of the iteration: the dense coarse
// operator A_c = R A P (App. A, "(R A P)"; Table 1 step 5), its LU
// factorisation with partial pivoting and its inverse, and y = A_c^{-1} x.
//
// The paper factors A_c with a direct LU (Sec. 4, PETSc).  Here the LU is a
// blocked right-looking getrf on the GPU; the per-iteration coarse solve then
// uses the explicit inverse (computed once from the LU factors by blocked
// triangular solves), which turns two sequential triangular sweeps into one
// bandwidth-bound, fully parallel matrix-vector product.
//
// All dense matrices are column-major with leading dimension n.
#include <algorithm>
#include <climits>
#include <vector>

#include "internal.hpp"

namespace fams {
namespace {

constexpr int kNb = 32;  // panel width of the blocked LU

// ---- A_c = R A P ------------------------------------------------------------
// One wavefront per coarse row I: walk the row of R (fine rows i ascending),
// the row of A, and the row of P; lanes own distinct coarse columns of one P
// row, rows are walked sequentially, so every sum has a fixed order.
__global__ void __launch_bounds__(64)
k_rap(int nc, const int* R_rp, const int* R_ci, const double* R_val, const int* rp,
      const int* ci, const double* av, const int* p_rp, const int* p_ci, const double* p_val,
      double* out, int jt) {
  extern __shared__ double acc[];
  const int I = blockIdx.x;
  const int lane = threadIdx.x;
  for (int j0 = 0; j0 < nc; j0 += jt) {
    const int j1 = min(nc, j0 + jt);
    for (int t = lane; t < j1 - j0; t += 64) acc[t] = 0.0;
    __syncthreads();
    for (int e = R_rp[I]; e < R_rp[I + 1]; ++e) {
      const int i = R_ci[e];
      const double w = R_val ? R_val[e] : 1.0;
      for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int j = ci[p];
        const double wa = w * av[p];
        for (int q = p_rp[j] + lane; q < p_rp[j + 1]; q += 64) {
          const int J = p_ci[q];
          if (J >= j0 && J < j1) acc[J - j0] += wa * p_val[q];
        }
        __syncthreads();
      }
    }
    for (int t = lane; t < j1 - j0; t += 64) out[static_cast<int64_t>(j0 + t) * nc + I] = acc[t];
    __syncthreads();
  }
}

// ---- A P, then A_c = R (A P) -------------------------------------------------
// Row i of A P = sum_j A_ij P_j, accumulated in A's column order into an LDS
// hash table of coarse columns (one wavefront per row, lanes over the
// entries of P_j, which have distinct columns).  Each row of A P is built once
// and reused by every coarse row whose restriction row contains i.
constexpr int kApSlots = 1024;   // hash slots per row (at most half used)
constexpr int kApWaves = 4;      // rows per 256-thread block
constexpr int kApEmpty = INT_MIN;
constexpr int kApSrc = 8;        // entries of a row of A whose P rows are loaded together

__device__ __forceinline__ int ap_slot(int* tab, int key, bool* full) {
  unsigned hh = (static_cast<unsigned>(key) * 2654435761u) & (kApSlots - 1);
  for (int probe = 0; probe < kApSlots; ++probe) {
    const int prev = atomicCAS(&tab[hh], kApEmpty, key);
    if (prev == kApEmpty || prev == key) return static_cast<int>(hh);
    hh = (hh + 1) & (kApSlots - 1);
  }
  *full = true;
  return -1;
}

// count (fill == false) or write (fill == true) the entries of rows of A P
template <bool kFill>
__global__ void __launch_bounds__(64 * kApWaves)
k_ap(int n, const int* rp, const int* ci, const double* av, const int* p_rp, const int* p_ci,
     const double* p_val, int64_t* cnt_or_ptr, int* ap_ci, double* ap_val, int* err) {
  __shared__ int tab[kApWaves][kApSlots];
  __shared__ double acc[kFill ? kApWaves : 1][kFill ? kApSlots : 1];
  __shared__ int s_cnt[kApWaves];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int i = blockIdx.x * kApWaves + wave;
  int* t = tab[wave];
  for (int k = lane; k < kApSlots; k += 64) {
    t[k] = kApEmpty;
    if constexpr (kFill) acc[wave][k] = 0.0;
  }
  if (lane == 0) s_cnt[wave] = 0;
  __syncthreads();
  bool full = false;
  if (i < n) {
    // kApSrc entries of A's row at a time: their P rows are loaded together
    // (lanes over a P row's entries, one register slot per entry of A), then
    // entered into the row's table in A's column order
    const int p0 = rp[i], p1 = rp[i + 1];
    for (int pb = p0; pb < p1; pb += kApSrc) {
      const int ps = pb + lane;
      const bool oks = lane < kApSrc && ps < p1;
      const int js = oks ? ci[ps] : 0;
      const double as = oks ? av[ps] : 0.0;
      const int qs = oks ? p_rp[js] : 0, qe = oks ? p_rp[js + 1] : 0;
      int key[kApSrc];
      double pv[kApSrc];
#pragma unroll
      for (int e = 0; e < kApSrc; ++e) {
        const int q = __shfl(qs, e) + lane;
        const bool ok = q < __shfl(qe, e);
        key[e] = ok ? p_ci[q] : kApEmpty;
        pv[e] = ok ? p_val[q] : 0.0;
      }
#pragma unroll
      for (int e = 0; e < kApSrc; ++e) {
        const double a = __shfl(as, e);
        if (key[e] != kApEmpty) {
          const int sl = ap_slot(t, key[e], &full);
          if constexpr (kFill) {
            if (sl >= 0) acc[wave][sl] += a * pv[e];
          }
        }
        const int qe_e = __shfl(qe, e);
        for (int q = __shfl(qs, e) + 64 + lane; q < qe_e; q += 64) {  // P rows beyond 64 entries
          const int sl = ap_slot(t, p_ci[q], &full);
          if constexpr (kFill) {
            if (sl >= 0) acc[wave][sl] += a * p_val[q];
          }
        }
      }
    }
  }
  __syncthreads();
  if (i < n) {
    int used = 0;
    for (int k = lane; k < kApSlots; k += 64) used += t[k] != kApEmpty;
    for (int off = 32; off > 0; off >>= 1) used += __shfl_xor(used, off);
    if (full || used > kApSlots / 2) {
      if (lane == 0) atomicOr(err, 1);
    } else if constexpr (!kFill) {
      if (lane == 0) cnt_or_ptr[i] = used;
    } else {
      const int64_t base = cnt_or_ptr[i];
      for (int k = lane; k < kApSlots; k += 64) {
        if (t[k] != kApEmpty) {
          const int o = atomicAdd(&s_cnt[wave], 1);
          ap_ci[base + o] = t[k];
          ap_val[base + o] = acc[wave][k];
        }
      }
    }
  }
}

// A_c rows: one workgroup of kRapWaves wavefronts per coarse row I.  Wavefront
// w takes the w-th quarter of the restriction row's entries e in order and
// forms acc_w[J] = sum_e w_e (A P)_{i_e, J} in its own LDS copy (one
// wavefront's LDS accesses are ordered, and the columns of one row of A P are
// distinct); the copies are then added in wavefront order, so every sum has a
// fixed order.
constexpr int kRapWaves = 4;
constexpr int kRapGroup = 8;  // entries of R whose rows of A P are loaded together

__global__ void __launch_bounds__(64 * kRapWaves)
k_rap_ap(int nc, const int* R_rp, const int* R_ci, const double* R_val, const int64_t* ap_rp,
         const int* ap_ci, const double* ap_val, double* out, int jt) {
  extern __shared__ double acc_all[];
  const int I = blockIdx.x;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  double* acc = acc_all + static_cast<int64_t>(wave) * jt;
  const int e0 = R_rp[I], e1 = R_rp[I + 1], ne = e1 - e0;
  const int eb = e0 + static_cast<int>(static_cast<int64_t>(ne) * wave / kRapWaves);
  const int ee = e0 + static_cast<int>(static_cast<int64_t>(ne) * (wave + 1) / kRapWaves);
  for (int j0 = 0; j0 < nc; j0 += jt) {
    const int j1 = min(nc, j0 + jt);
    for (int t = lane; t < j1 - j0; t += 64) acc[t] = 0.0;
    // kRapGroup entries of R at a time: their bounds (lanes), then the first
    // 64 entries of each of their rows of A P are loaded together and added
    // in R's order
    for (int e0b = eb; e0b < ee; e0b += kRapGroup) {
      const int el = e0b + lane;
      const bool okl = lane < kRapGroup && el < ee;
      const int il = okl ? R_ci[el] : 0;
      const int64_t ql0 = okl ? ap_rp[il] : 0, ql1 = okl ? ap_rp[il + 1] : 0;
      const double wl = okl ? (R_val ? R_val[el] : 1.0) : 0.0;
      int Jv[kRapGroup];
      double v[kRapGroup];
#pragma unroll
      for (int g = 0; g < kRapGroup; ++g) {
        const int64_t q = __shfl(ql0, g) + lane;
        const bool ok = q < __shfl(ql1, g);
        Jv[g] = ok ? ap_ci[q] : -1;
        v[g] = ok ? ap_val[q] : 0.0;
      }
#pragma unroll
      for (int g = 0; g < kRapGroup; ++g) {
        const double w = __shfl(wl, g);
        if (Jv[g] >= j0 && Jv[g] < j1) acc[Jv[g] - j0] += w * v[g];
        const int64_t q1 = __shfl(ql1, g);
        for (int64_t q = __shfl(ql0, g) + 64 + lane; q < q1; q += 64) {  // rows beyond 64 entries
          const int J = ap_ci[q];
          if (J >= j0 && J < j1) acc[J - j0] += w * ap_val[q];
        }
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < j1 - j0; t += blockDim.x) {
      double v = acc_all[t];
      for (int k = 1; k < kRapWaves; ++k) v += acc_all[static_cast<int64_t>(k) * jt + t];
      out[static_cast<int64_t>(j0 + t) * nc + I] = v;
    }
    __syncthreads();
  }
}

// The same rows in one pass over R's entries: the coarse row's columns J go
// into an LDS hash table shared by the workgroup's wavefronts (kRapSlots
// keys; a wavefront's instruction holds distinct columns, and every
// wavefront has its own value copy), each wavefront adds its quarter of the
// entries in R's order, and the copies are added in wavefront order, so
// every sum is the one k_rap_ap forms.  k_rap_ap keeps a dense accumulator
// per wavefront, at most jt columns wide for LDS, and so reads R's entries
// and their rows of A P once per jt columns (five times at n_c = 17,810).
// `out` must hold zeros; a row with more than kRapSlots / 2 distinct columns
// sets *err and writes nothing (the caller then uses k_rap_ap).
constexpr int kRapSlots = 2048;

__device__ __forceinline__ int rap_slot(int* tab, int key, bool* full) {
  unsigned hh = (static_cast<unsigned>(key) * 2654435761u) & (kRapSlots - 1);
  for (int probe = 0; probe < kRapSlots; ++probe) {
    const int prev = atomicCAS(&tab[hh], kApEmpty, key);
    if (prev == kApEmpty || prev == key) return static_cast<int>(hh);
    hh = (hh + 1) & (kRapSlots - 1);
  }
  *full = true;
  return -1;
}

__global__ void __launch_bounds__(64 * kRapWaves)
k_rap_hash(int nc, const int* R_rp, const int* R_ci, const double* R_val, const int64_t* ap_rp,
           const int* ap_ci, const double* ap_val, double* out, int* err) {
  __shared__ int keys[kRapSlots];
  __shared__ double acc[kRapWaves][kRapSlots];
  __shared__ int s_bad, s_used;
  const int I = blockIdx.x;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  for (int k = threadIdx.x; k < kRapSlots; k += blockDim.x) {
    keys[k] = kApEmpty;
#pragma unroll
    for (int w = 0; w < kRapWaves; ++w) acc[w][k] = 0.0;
  }
  if (threadIdx.x == 0) s_bad = s_used = 0;
  __syncthreads();
  const int e0 = R_rp[I], e1 = R_rp[I + 1], ne = e1 - e0;
  const int eb = e0 + static_cast<int>(static_cast<int64_t>(ne) * wave / kRapWaves);
  const int ee = e0 + static_cast<int>(static_cast<int64_t>(ne) * (wave + 1) / kRapWaves);
  double* a = acc[wave];
  bool full = false;
  for (int e0b = eb; e0b < ee; e0b += kRapGroup) {
    const int el = e0b + lane;
    const bool okl = lane < kRapGroup && el < ee;
    const int il = okl ? R_ci[el] : 0;
    const int64_t ql0 = okl ? ap_rp[il] : 0, ql1 = okl ? ap_rp[il + 1] : 0;
    const double wl = okl ? (R_val ? R_val[el] : 1.0) : 0.0;
    int Jv[kRapGroup];
    double v[kRapGroup];
#pragma unroll
    for (int g = 0; g < kRapGroup; ++g) {
      const int64_t q = __shfl(ql0, g) + lane;
      const bool ok = q < __shfl(ql1, g);
      Jv[g] = ok ? ap_ci[q] : -1;
      v[g] = ok ? ap_val[q] : 0.0;
    }
#pragma unroll
    for (int g = 0; g < kRapGroup; ++g) {
      const double w = __shfl(wl, g);
      if (Jv[g] >= 0) {
        const int sl = rap_slot(keys, Jv[g], &full);
        if (sl >= 0) a[sl] += w * v[g];
      }
      const int64_t q1 = __shfl(ql1, g);
      for (int64_t q = __shfl(ql0, g) + 64 + lane; q < q1; q += 64) {  // rows beyond 64 entries
        const int sl = rap_slot(keys, ap_ci[q], &full);
        if (sl >= 0) a[sl] += w * ap_val[q];
      }
    }
  }
  if (full) atomicOr(&s_bad, 1);
  __syncthreads();
  int used = 0;
  for (int k = threadIdx.x; k < kRapSlots; k += blockDim.x) used += keys[k] != kApEmpty;
  atomicAdd(&s_used, used);
  __syncthreads();
  if (s_bad || s_used > kRapSlots / 2) {
    if (threadIdx.x == 0) atomicOr(err, 1);
    return;
  }
  for (int k = threadIdx.x; k < kRapSlots; k += blockDim.x) {
    if (keys[k] == kApEmpty) continue;
    double t = acc[0][k];
#pragma unroll
    for (int w = 1; w < kRapWaves; ++w) t += acc[w][k];
    out[static_cast<int64_t>(keys[k]) * nc + I] = t;
  }
}

// ---- LU with partial pivoting ----------------------------------------------
// Panel [k0, k0+nb) of rows [k0, n): pivot = first row of maximal |a|.
__global__ void __launch_bounds__(1024)
k_panel(double* a, int n, int k0, int nb, int* ipiv, int* info) {
  __shared__ double s_val[1024];
  __shared__ int s_idx[1024];
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  for (int j = k0; j < k0 + nb; ++j) {
    double* colj = a + static_cast<int64_t>(j) * n;
    double best = -1.0;
    int bi = n;
    for (int r = j + tid; r < n; r += nt) {
      double v = fabs(colj[r]);
      if (v > best) {
        best = v;
        bi = r;
      }
    }
    s_val[tid] = best;
    s_idx[tid] = bi;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
      if (tid < s) {
        double v2 = s_val[tid + s];
        int i2 = s_idx[tid + s];
        if (v2 > s_val[tid] || (v2 == s_val[tid] && i2 < s_idx[tid])) {
          s_val[tid] = v2;
          s_idx[tid] = i2;
        }
      }
      __syncthreads();
    }
    const int piv = s_idx[0];
    const double pval = s_val[0];
    __syncthreads();
    if (tid == 0) {
      ipiv[j] = piv;
      if (!(pval > 0.0) && *info == 0) *info = j + 1;
    }
    if (piv != j) {
      for (int c = k0 + tid; c < k0 + nb; c += nt) {
        double* cc = a + static_cast<int64_t>(c) * n;
        double t = cc[j];
        cc[j] = cc[piv];
        cc[piv] = t;
      }
    }
    __syncthreads();
    const double d = colj[j];
    const double rd = d != 0.0 ? 1.0 / d : 0.0;
    for (int r = j + 1 + tid; r < n; r += nt) colj[r] *= rd;
    __syncthreads();
    const int w = k0 + nb - (j + 1);
    const int64_t rows = n - (j + 1);
    for (int64_t idx = tid; idx < rows * w; idx += nt) {
      int c = j + 1 + static_cast<int>(idx / rows);
      int r = j + 1 + static_cast<int>(idx % rows);
      double* cc = a + static_cast<int64_t>(c) * n;
      cc[r] -= colj[r] * cc[j];
    }
    __syncthreads();
  }
}

// One step of the wavefront argmax below: every lane enabled by kRowMask
// combines its candidate with the one the DPP pattern kCtrl routes to it
// (lanes without a source keep their own).  Larger |a| wins, then the lower
// position: a total order, so the combining order does not matter.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ void argmax_dpp(double& v, int& p) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const int lo = static_cast<int>(static_cast<unsigned>(u));
  const int hi = static_cast<int>(static_cast<unsigned>(u >> 32));
  const int olo = __builtin_amdgcn_update_dpp(lo, lo, kCtrl, kRowMask, 0xf, false);
  const int ohi = __builtin_amdgcn_update_dpp(hi, hi, kCtrl, kRowMask, 0xf, false);
  const int op = __builtin_amdgcn_update_dpp(p, p, kCtrl, kRowMask, 0xf, false);
  const double ov = __builtin_bit_cast(
      double, (static_cast<unsigned long long>(static_cast<unsigned>(ohi)) << 32) |
                  static_cast<unsigned>(olo));
  if (ov > v || (ov == v && op < p)) {
    v = ov;
    p = op;
  }
}

// (max |a|, its lowest position) over the wavefront, in every lane: an
// inclusive scan within each row of 16 lanes (row_shr 1, 2, 4, 8), then the
// last lane of a row is passed on to the next rows (row_bcast 15 and 31),
// which leaves the whole wavefront's result in lane 63.
__device__ __forceinline__ void wave_argmax(double& v, int& p) {
  argmax_dpp<0x111, 0xf>(v, p);  // row_shr:1
  argmax_dpp<0x112, 0xf>(v, p);  // row_shr:2
  argmax_dpp<0x114, 0xf>(v, p);  // row_shr:4
  argmax_dpp<0x118, 0xf>(v, p);  // row_shr:8
  argmax_dpp<0x142, 0xa>(v, p);  // row_bcast:15 into rows 1 and 3
  argmax_dpp<0x143, 0xc>(v, p);  // row_bcast:31 into rows 2 and 3
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = static_cast<unsigned>(
      __builtin_amdgcn_readlane(static_cast<int>(static_cast<unsigned>(u)), 63));
  const unsigned hi = static_cast<unsigned>(
      __builtin_amdgcn_readlane(static_cast<int>(static_cast<unsigned>(u >> 32)), 63));
  v = __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
  p = __builtin_amdgcn_readlane(p, 63);
}

// Panel of nb <= 16 columns held in registers (rows [k0, n), at most 512*RT
// of them; thread t owns rows t, t+512, ...).  Row interchanges are logical:
// pos[] is each row's current position and at_pos[] its inverse, so a step
// costs two barriers and no memory traffic; the rows are written back to
// their final positions at the end.  Pivot choice (first maximal |a| in
// position order) and every update are the same as in k_panel.
//
// With kpn > 0 the kernel first applies the previous panel (columns
// [k0 - kpn, k0), already factored) to its own columns, as the separate
// launches would: that panel's interchanges (as a row map built in LDS, so
// the columns are read once, through it), the unit lower triangular solve
// for rows [k0 - kpn, k0) (written back: they are rows of U), then
// the update of rows [k0, n) by L21 U12 while the panel is loaded.
constexpr int kRegNb = 16;
constexpr int kRegThreads = 512;

template <int RT>
__global__ void __launch_bounds__(kRegThreads)
k_panel_reg(double* a, int n, int k0, int nb, int* ipiv, int* info, int kpn) {
  __shared__ int at_pos[kRegThreads * RT];
  __shared__ double s_best[kRegThreads / 64];
  __shared__ int s_bpos[kRegThreads / 64];
  __shared__ double s_prow[kRegNb];
  __shared__ int s_src[kRegThreads * RT + kRegNb];  // row map of [k0 - kpn, n)
  __shared__ double s_u[kRegNb * kRegNb];           // U12: [row j][column c]
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int m = n - k0, kp0 = k0 - kpn;
  if (kpn > 0) {
    for (int l = tid; l < m + kpn; l += kRegThreads) s_src[l] = l;
    __syncthreads();
    if (tid == 0) {  // the previous panel's interchanges, in order
      int pv[kRegNb];
#pragma clang loop unroll(full)
      for (int j = 0; j < kRegNb; ++j)
        if (j < kpn) pv[j] = ipiv[kp0 + j] - kp0;
#pragma clang loop unroll(full)
      for (int j = 0; j < kRegNb; ++j)
        if (j < kpn && pv[j] != j) {
          const int t = s_src[j];
          s_src[j] = s_src[pv[j]];
          s_src[pv[j]] = t;
        }
    }
    __syncthreads();
  }
  // every old value is read before the U rows of the previous panel are
  // written (a row of [k0 - kpn, k0) may be the source of a row below)
  double x[kRegNb];
  if (kpn > 0 && tid < nb) {
    const double* cc = a + static_cast<int64_t>(k0 + tid) * n + kp0;
#pragma clang loop unroll(full)
    for (int j = 0; j < kRegNb; ++j) x[j] = j < kpn ? cc[s_src[j]] : 0.0;
  }
  double v[RT][kRegNb];
  int pos[RT];
#pragma clang loop unroll(full)
  for (int q = 0; q < RT; ++q) {
    const int r = tid + q * kRegThreads;
    pos[q] = r < m ? r : INT_MAX;
    const int src = r < m ? (kpn > 0 ? s_src[kpn + r] : r) : 0;
#pragma clang loop unroll(full)
    for (int c = 0; c < kRegNb; ++c)
      v[q][c] = (r < m && c < nb) ? a[static_cast<int64_t>(k0 + c) * n + kp0 + src] : 0.0;
    if (r < m) at_pos[r] = r;
  }
  __syncthreads();
  if (kpn > 0) {
    if (tid < nb) {  // U12 column k0 + tid: unit lower solve with L11
      const double* l11 = a + static_cast<int64_t>(kp0) * n + kp0;
#pragma clang loop unroll(full)
      for (int r = 1; r < kRegNb; ++r)
        if (r < kpn) {
          double s = x[r];
#pragma clang loop unroll(full)
          for (int t = 0; t < r; ++t) s -= l11[static_cast<int64_t>(t) * n + r] * x[t];
          x[r] = s;
        }
      double* cc = a + static_cast<int64_t>(k0 + tid) * n + kp0;
#pragma clang loop unroll(full)
      for (int j = 0; j < kRegNb; ++j)
        if (j < kpn) {
          cc[j] = x[j];
          s_u[j * kRegNb + tid] = x[j];
        }
    }
    __syncthreads();
#pragma clang loop unroll(full)
    for (int q = 0; q < RT; ++q) {
      const int r = tid + q * kRegThreads;
      if (r < m) {
        double l[kRegNb];
#pragma clang loop unroll(full)
        for (int j = 0; j < kRegNb; ++j)
          l[j] = j < kpn ? a[static_cast<int64_t>(kp0 + j) * n + k0 + r] : 0.0;
#pragma clang loop unroll(full)
        for (int c = 0; c < kRegNb; ++c) {
          if (c >= nb) continue;
          double acc = 0.0;
#pragma clang loop unroll(full)
          for (int j = 0; j < kRegNb; ++j)
            if (j < kpn) acc += l[j] * s_u[j * kRegNb + c];
          v[q][c] -= acc;
        }
      }
    }
  }
#pragma clang loop unroll(full)
  for (int j = 0; j < kRegNb; ++j) {
    if (j < nb) {
    double best = -1.0;
    int bpos = INT_MAX;
#pragma clang loop unroll(full)
    for (int q = 0; q < RT; ++q) {
      if (pos[q] >= j && pos[q] != INT_MAX) {
        const double x = fabs(v[q][j]);
        if (x > best || (x == best && pos[q] < bpos)) {
          best = x;
          bpos = pos[q];
        }
      }
    }
    wave_argmax(best, bpos);
    if (lane == 0) {
      s_best[wave] = best;
      s_bpos[wave] = bpos;
    }
    __syncthreads();
    double pval = s_best[0];
    int ppos = s_bpos[0];
    for (int w = 1; w < kRegThreads / 64; ++w) {
      if (s_best[w] > pval || (s_best[w] == pval && s_bpos[w] < ppos)) {
        pval = s_best[w];
        ppos = s_bpos[w];
      }
    }
    const int prow = at_pos[ppos], jrow = at_pos[j];
#pragma clang loop unroll(full)
    for (int q = 0; q < RT; ++q) {
      if (tid + q * kRegThreads == prow) {
#pragma clang loop unroll(full)
        for (int c = 0; c < kRegNb; ++c) s_prow[c] = v[q][c];
      }
    }
    __syncthreads();
    if (tid == 0) {
      ipiv[k0 + j] = k0 + ppos;
      if (!(pval > 0.0) && *info == 0) *info = k0 + j + 1;
      at_pos[j] = prow;
      at_pos[ppos] = jrow;
    }
#pragma clang loop unroll(full)
    for (int q = 0; q < RT; ++q) {
      const int r = tid + q * kRegThreads;
      if (r == prow) pos[q] = j;
      else if (r == jrow) pos[q] = ppos;
    }
    const double d = s_prow[j];
    const double rd = d != 0.0 ? 1.0 / d : 0.0;
#pragma clang loop unroll(full)
    for (int q = 0; q < RT; ++q) {
      if (pos[q] > j && pos[q] != INT_MAX) {
        const double l = v[q][j] * rd;
        v[q][j] = l;
#pragma clang loop unroll(full)
        for (int c = j + 1; c < kRegNb; ++c) v[q][c] -= l * s_prow[c];
      }
    }
  }
  }
#pragma clang loop unroll(full)
  for (int q = 0; q < RT; ++q) {
    if (pos[q] != INT_MAX) {
#pragma clang loop unroll(full)
      for (int c = 0; c < kRegNb; ++c)
        if (c < nb) a[static_cast<int64_t>(k0 + c) * n + k0 + pos[q]] = v[q][c];
    }
  }
}


// B[k0:k0+nb, c] <- L11^{-1} B[...] (unit lower L11 at (k0, k0) of `l`), for
// columns c in [c0, c1) of `b`; one thread per column
__global__ void k_trsm_lower_unit(const double* l, int n, int k0, int nb, double* b, int c0,
                                  int c1) {
  __shared__ double L[kNb * kNb];
  for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
    int r = t % nb, c = t / nb;
    L[t] = l[static_cast<int64_t>(k0 + c) * n + k0 + r];
  }
  __syncthreads();
  int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= c1) return;
  double x[kNb];
  double* col = b + static_cast<int64_t>(c) * n + k0;
  for (int r = 0; r < nb; ++r) x[r] = col[r];
  for (int r = 0; r < nb; ++r) {
    double s = x[r];
    for (int t = 0; t < r; ++t) s -= L[t * nb + r] * x[t];
    x[r] = s;
  }
  for (int r = 0; r < nb; ++r) col[r] = x[r];
}

// the panel's row interchanges applied to the columns [lo1, lo1 + n1) and
// [lo2, lo2 + n2) (none of them in the panel), then, for those after the
// panel, B[k0:k0+nb, c] <- L11^{-1} B[...] (unit lower L11 of the factored
// panel); one thread per column
__global__ void k_swap_trsm(double* a, int n, int k0, int nb, const int* ipiv, int lo1, int n1,
                            int lo2, int n2) {
  __shared__ double L[kNb * kNb];
  for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
    int r = t % nb, c = t / nb;
    L[t] = a[static_cast<int64_t>(k0 + c) * n + k0 + r];
  }
  __syncthreads();
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n1 + n2) return;
  const int c = t < n1 ? lo1 + t : lo2 + (t - n1);
  double* cc = a + static_cast<int64_t>(c) * n;
  for (int j = k0; j < k0 + nb; ++j) {
    int p = ipiv[j];
    if (p != j) {
      double t = cc[j];
      cc[j] = cc[p];
      cc[p] = t;
    }
  }
  if (c < k0 + nb) return;
  double x[kNb];
  double* col = cc + k0;
  for (int r = 0; r < nb; ++r) x[r] = col[r];
  for (int r = 0; r < nb; ++r) {
    double s = x[r];
    for (int t = 0; t < r; ++t) s -= L[t * nb + r] * x[t];
    x[r] = s;
  }
  for (int r = 0; r < nb; ++r) col[r] = x[r];
}

// B[k0:k0+nb, c] <- U11^{-1} B[...] (upper, non-unit U11 at (k0, k0) of `u`)
__global__ void k_trsm_upper(const double* u, int n, int k0, int nb, double* b, int c0, int c1) {
  __shared__ double U[kNb * kNb];
  for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
    int r = t % nb, c = t / nb;
    U[t] = u[static_cast<int64_t>(k0 + c) * n + k0 + r];
  }
  __syncthreads();
  int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= c1) return;
  double x[kNb];
  double* col = b + static_cast<int64_t>(c) * n + k0;
  for (int r = 0; r < nb; ++r) x[r] = col[r];
  for (int r = nb - 1; r >= 0; --r) {
    double s = x[r];
    for (int t = r + 1; t < nb; ++t) s -= U[t * nb + r] * x[t];
    x[r] = s / U[r * nb + r];
  }
  for (int r = 0; r < nb; ++r) col[r] = x[r];
}

__global__ void k_perm_identity(int n, const int* perm, double* x) {
  int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<int64_t>(n) * n) return;
  int r = static_cast<int>(t % n), c = static_cast<int>(t / n);
  x[t] = perm[r] == c ? 1.0 : 0.0;
}

// y = M x, M column-major n x n: partial sums over column chunks, then a
// fixed-order reduction across chunks
constexpr int kGemvChunk = 64;
__global__ void k_gemv_part(int n, const double* M, const double* x, double* part) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  int c0 = blockIdx.y * kGemvChunk;
  if (I >= n) return;
  int c1 = min(n, c0 + kGemvChunk);
  double s = 0.0;
  for (int c = c0; c < c1; ++c) s += M[static_cast<int64_t>(c) * n + I] * x[c];
  part[static_cast<int64_t>(blockIdx.y) * n + I] = s;
}

__global__ void k_gemv_reduce(int n, int nchunks, const double* part, double* y) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= n) return;
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += part[static_cast<int64_t>(c) * n + I];
  y[I] = s;
}

void gemm_mfma(Handle* h, int m, int p, int k, double alpha, const double* A, int lda,
               const double* B, int ldb, double* C, int ldc, int skip0 = 0, int skip1 = 0,
               hipStream_t st = nullptr, bool overwrite = false);

// C[m x p] -= A[m x k] B[k x p] (common leading dimension) on FP64 MFMA
void gemm_sub(Handle* h, int m, int p, int k, const double* A, const double* B, double* C,
              int ld, hipStream_t st = nullptr) {
  gemm_mfma(h, m, p, k, -1.0, A, ld, B, ld, C, ld, 0, 0, st);
}

// ---- FP64 MFMA GEMM ----------------------------------------------------------
// C[r, c] += alpha * sum_q A[r, q] B[q, c] for r < m, c < p, except rows and
// columns in [skip0, skip1); column-major operands.  A workgroup forms a
// 64 x 64 tile, each wavefront a 32 x 32 quarter of 2 x 2 blocks of
// v_mfma_f64_16x16x4 (per instruction lane l supplies A[l%16][l/16] and
// B[l/16][l%16] and holds D[4*q + l/16][l%16] in accumulator element q).
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kGT = 64, kGK = 16;

__global__ void __launch_bounds__(256)
k_gemm_mfma(int m, int p, int k, double alpha, const double* A, int lda, const double* B,
            int ldb, double* C, int ldc, int skip0, int skip1, int overwrite) {
  __shared__ double As[kGK][kGT + 1];
  __shared__ double Bs[kGK][kGT + 1];
  const int r0 = blockIdx.x * kGT, c0 = blockIdx.y * kGT;
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int wr = (wave % 2) * 32, wc = (wave / 2) * 32;
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < k; k0 += kGK) {
    for (int e = tid; e < kGK * kGT; e += 256) {
      const int i = e % kGT, qa = e / kGT;
      As[qa][i] = (r0 + i < m && k0 + qa < k) ? A[static_cast<int64_t>(k0 + qa) * lda + r0 + i] : 0.0;
      const int qb = e % kGK, j = e / kGK;
      Bs[qb][j] = (c0 + j < p && k0 + qb < k) ? B[static_cast<int64_t>(c0 + j) * ldb + k0 + qb] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 4) {
      double fa[2], fb[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        fa[t] = As[kk + lane / 16][wr + t * 16 + lane % 16];
        fb[t] = Bs[kk + lane / 16][wc + t * 16 + lane % 16];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + wr + a * 16 + 4 * q + lane / 16;
        const int c = c0 + wc + b * 16 + lane % 16;
        if (r < m && c < p && (r < skip0 || r >= skip1) && (c < skip0 || c >= skip1)) {
          double* o = C + static_cast<int64_t>(c) * ldc + r;
          *o = overwrite ? alpha * acc[a][b][q] : *o + alpha * acc[a][b][q];
        }
      }
}

// Large-tile form: a workgroup of eight wavefronts forms a 128 x 128 tile,
// each wavefront a 64 x 32 eighth of 4 x 2 blocks of v_mfma_f64_16x16x4
// (8 accumulators of four doubles); two wavefronts per SIMD, so one's load
// and address work overlaps the other's MFMAs.  The k dimension advances
// kBK at a time through two LDS buffers: while the MFMAs consume one
// buffer, every thread holds the next kBK-wide slices of A and B in
// registers (loaded from clamped addresses, zeroed outside the operands,
// without branches) and stores them into the other buffer after the step,
// so one barrier per step and the global loads overlap the arithmetic.
// Tiles are numbered in a one-dimensional grid: workgroups go to the eight
// XCDs in turn (b % 8), each XCD takes a contiguous run of the tile order,
// and the order walks groups of kGroupRows row tiles column tile by column
// tile, so the tiles an XCD runs at once share A's rows and B's columns in
// its L2 (with the workgroups of a column of tiles spread over all XCDs,
// every XCD streamed every operand tile from beyond its L2).
constexpr int kBT = 128, kBK = 32, kBPad = kBT + 4, kGroupRows = 8;

__device__ __forceinline__ void gemm_tile(int tr_n, int tc_n, int& tr, int& tc) {
  const int T = tr_n * tc_n, b = blockIdx.x;
  const int x = b % kXcd, s = b / kXcd;
  const int g = x * (T / kXcd) + min(x, T % kXcd) + s;
  const int span = kGroupRows * tc_n;
  const int first = (g / span) * kGroupRows;
  const int rows = min(kGroupRows, tr_n - first);
  const int o = g - (g / span) * span;
  tr = first + o % rows;
  tc = o / rows;
}

constexpr int kBThreads = 512, kBWc = 2;  // threads, column blocks per wavefront

__global__ void __launch_bounds__(kBThreads)
k_gemm_mfma128(int m, int p, int k, double alpha, const double* A, int lda, const double* B,
               int ldb, double* C, int ldc, int skip0, int skip1, int overwrite) {
  __shared__ double As[2][kBK][kBPad];
  __shared__ double Bs[2][kBK][kBPad];
  int tr, tc;
  gemm_tile((m + kBT - 1) / kBT, (p + kBT - 1) / kBT, tr, tc);
  const int r0 = tr * kBT, c0 = tc * kBT;
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int wr = (wave % 2) * 64, wc = (wave / 2) * (16 * kBWc);
  // global slice loads: A column-major, 128 rows x kBK k: thread t loads row
  // t % 128 at k = t / 128 + 4u; B column-major, kBK k x 128 columns: thread t
  // loads k = t % kBK of columns t / kBK + (512 / kBK) u; kBK / 4 of each
  constexpr int kL = kBK * kBT / kBThreads, kAs = kBThreads / kBT, kCs = kBThreads / kBK;
  const int ar = tid % kBT, ak = tid / kBT;
  const int bk = tid % kBK, bc = tid / kBK;
  double ra[kL], rb[kL];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < kL; ++u) {
      const int kk = k0 + ak + kAs * u, rr = r0 + ar;
      const bool oa = rr < m && kk < k;
      const double va = A[oa ? static_cast<int64_t>(kk) * lda + rr : 0];
      ra[u] = oa ? va : 0.0;
      const int kb = k0 + bk, cc = c0 + bc + kCs * u;
      const bool ob = cc < p && kb < k;
      const double vb = B[ob ? static_cast<int64_t>(cc) * ldb + kb : 0];
      rb[u] = ob ? vb : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < kL; ++u) {
      As[buf][ak + kAs * u][ar] = ra[u];
      Bs[buf][bk][bc + kCs * u] = rb[u];
    }
  };
  v4d acc[4][kBWc];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < kBWc; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  load(0);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < k; k0 += kBK) {
    const bool more = k0 + kBK < k;
    if (more) load(k0 + kBK);
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 4) {
      double fa[4], fb[kBWc];
#pragma unroll
      for (int t = 0; t < 4; ++t) fa[t] = As[buf][kk + lane / 16][wr + t * 16 + lane % 16];
#pragma unroll
      for (int t = 0; t < kBWc; ++t) fb[t] = Bs[buf][kk + lane / 16][wc + t * 16 + lane % 16];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < kBWc; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < kBWc; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + wr + a * 16 + 4 * q + lane / 16;
        const int c = c0 + wc + b * 16 + lane % 16;
        if (r < m && c < p && (r < skip0 || r >= skip1) && (c < skip0 || c >= skip1)) {
          double* o = C + static_cast<int64_t>(c) * ldc + r;
          *o = overwrite ? alpha * acc[a][b][q] : *o + alpha * acc[a][b][q];
        }
      }
}

void gemm_mfma(Handle* h, int m, int p, int k, double alpha, const double* A, int lda,
               const double* B, int ldb, double* C, int ldc, int skip0, int skip1,
               hipStream_t st, bool overwrite) {
  if (m <= 0 || p <= 0 || k <= 0) return;
  hipStream_t s = st ? st : h->stream;
  const int ow = overwrite ? 1 : 0;
  if (static_cast<int64_t>(blocks_for(m, kBT)) * blocks_for(p, kBT) >= 192) {
    const unsigned tiles = blocks_for(m, kBT) * blocks_for(p, kBT);
    LAUNCH_ON(h, s, "gemm_mfma", k_gemm_mfma128, tiles, kBThreads, 0, m, p, k, alpha, A, lda, B,
              ldb, C, ldc, skip0, skip1, ow);
  } else {  // small products: more, smaller tiles keep the device busy
    dim3 grid(blocks_for(m, kGT), blocks_for(p, kGT));
    LAUNCH_ON(h, s, "gemm_mfma", k_gemm_mfma, grid, 256, 0, m, p, k, alpha, A, lda, B, ldb, C,
              ldc, skip0, skip1, ow);
  }
}

// ---- in-place Gauss-Jordan inverse by blocks (no pivoting; SPD A_c) ---------
// Step k with B = block k: B B <- inv(B B); column block <- -(column block)
// inv(B B); every other entry += (new column block)(old row block); row block
// <- inv(B B)(row block).  2 n^3 flops, the rank-kNb updates on MFMA.
__global__ void __launch_bounds__(1024) k_gje_block(double* a, int n, int k0, int nb, int* info) {
  __shared__ double T[kNb][kNb + 1];
  const int i = threadIdx.x % kNb, c = threadIdx.x / kNb;
  const bool in = i < nb && c < nb;
  if (in) T[i][c] = a[static_cast<int64_t>(k0 + c) * n + k0 + i];
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    const double d = T[j][j];
    if (threadIdx.x == 0 && !(d > 0.0)) atomicCAS(info, 0, k0 + j + 1);
    const double rd = 1.0 / d;
    const double f = in ? T[i][j] : 0.0, rj = in ? T[j][c] : 0.0;
    __syncthreads();
    if (in) {
      double v;
      if (i == j && c == j) v = rd;
      else if (i == j) v = rj * rd;
      else if (c == j) v = -f * rd;
      else v = T[i][c] - f * (rj * rd);
      T[i][c] = v;
    }
    __syncthreads();
  }
  if (in) a[static_cast<int64_t>(k0 + c) * n + k0 + i] = T[i][c];
}

// column block rows r outside the block: a[r, blk] <- -a[r, blk] inv(B B).
// One thread per (row, output column); a workgroup covers 8 rows x 32
// columns and stages the 8 rows' old values before writing.
__global__ void __launch_bounds__(256) k_gje_col(double* a, int n, int k0, int nb) {
  __shared__ double T[kNb][kNb + 1];
  __shared__ double X[8][kNb + 1];
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x)
    T[e % nb][e / nb] = a[static_cast<int64_t>(k0 + e / nb) * n + k0 + e % nb];
  const int rl = threadIdx.x % 8, c = threadIdx.x / 8;   // 8 rows x 32 columns
  int r = blockIdx.x * 8 + rl;
  if (r >= k0) r += nb;                                     // skip the block's rows
  const bool in = r < n && c < nb;
  if (in) X[rl][c] = a[static_cast<int64_t>(k0 + c) * n + r];
  __syncthreads();
  if (!in) return;
  double s = 0.0;
  for (int q = 0; q < nb; ++q) s += X[rl][q] * T[q][c];
  a[static_cast<int64_t>(k0 + c) * n + r] = -s;
}

// row block columns c outside the block: a[blk, c] <- inv(B B) a[blk, c];
// one thread per (output row, column), 32 x 8 per workgroup
__global__ void __launch_bounds__(256) k_gje_row(double* a, int n, int k0, int nb) {
  __shared__ double T[kNb][kNb + 1];
  __shared__ double Y[8][kNb + 1];
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x)
    T[e % nb][e / nb] = a[static_cast<int64_t>(k0 + e / nb) * n + k0 + e % nb];
  const int i = threadIdx.x % kNb, cl = threadIdx.x / kNb;  // 32 rows x 8 columns
  int c = blockIdx.x * 8 + cl;
  if (c >= k0) c += nb;
  const bool in = c < n && i < nb;
  if (in) Y[cl][i] = a[static_cast<int64_t>(c) * n + k0 + i];
  __syncthreads();
  if (!in) return;
  double s = 0.0;
  for (int q = 0; q < nb; ++q) s += T[i][q] * Y[cl][q];
  a[static_cast<int64_t>(c) * n + k0 + i] = s;
}

// ---- solves with LU factors ---------------------------------------------------
// x = A^{-1} b from P A = L U (factors column-major): x <- P b, then L (unit)
// and U, each in one launch of one wavefront per chunk of 64 rows.  The
// wavefront of chunk i subtracts the contributions of the chunks before it
// (after it, for U) in chunk order, each as soon as that chunk's solution is
// published, then solves its 64 x 64 diagonal block with register shuffles,
// publishes its own solution and raises its flag.  Chunks wait only on
// chunks dispatched before them.  A wait is bounded (`limit` ticks): on
// timeout err is set, the remaining waits end at once and the result is void.
constexpr int kLuSolveMax = 1 << 20;
constexpr int kLuB = 64;

__global__ void k_gather_perm(int n, const int* perm, const double* b, double* w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = b[perm[i]];
}

template <bool kUpper>
__global__ void __launch_bounds__(64)
k_lu_df(int n, const double* lu, const double* w, double* x, int* flag, int epoch, int* err,
        int* ticket, unsigned long long limit) {
  const int lane = threadIdx.x;
  const int nch = (n + kLuB - 1) / kLuB;
  // chunks by ticket in solve order: every chunk this one waits for has been
  // taken by a workgroup already running, whatever order the hardware
  // dispatches the workgroups in
  __shared__ int s_t;
  if (lane == 0) s_t = atomicAdd(ticket, 1);
  __syncthreads();
  const int ci = kUpper ? nch - 1 - s_t : s_t;
  const int r0 = ci * kLuB, nbk = min(kLuB, n - r0), r = r0 + lane;
  const bool own = lane < nbk;
  double v = own ? w[r] : 0.0;
  auto wait = [&](int j) {
    const unsigned long long t0 = wall_clock64();
    while (true) {
      int f = __hip_atomic_load(flag + j, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
      f = __builtin_amdgcn_readfirstlane(f);
      if (f == epoch) {
        // waits beyond ~1 ms (limit / 2048) are counted in err[3]
        if (lane == 0 && wall_clock64() - t0 > (limit >> 11)) atomicAdd(err + 3, 1);
        break;
      }
      int e = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      e = __builtin_amdgcn_readfirstlane(e);
      if (e != 0) break;
      if (wall_clock64() - t0 > limit) {
        if (lane == 0) atomicOr(err, 1);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  };
  // contributions of the other chunks, in the order the chunks finish
  for (int s = 0; s < (kUpper ? nch - 1 - ci : ci); ++s) {
    const int j = kUpper ? nch - 1 - s : s;
    const int c0 = j * kLuB, nbj = min(kLuB, n - c0);
    double a[kLuB];
#pragma unroll
    for (int q = 0; q < kLuB; ++q)
      a[q] = (own && q < nbj) ? lu[static_cast<int64_t>(c0 + q) * n + r] : 0.0;
    wait(j);
    const double xj = lane < nbj ? x[c0 + lane] : 0.0;
#pragma unroll
    for (int q = 0; q < kLuB; ++q) {
      const double xq = __shfl(xj, q);
      if (q < nbj) v -= a[q] * xq;
    }
  }
  // the diagonal block: A(r0 + lane, r0 + q)
  double d[kLuB];
#pragma unroll
  for (int q = 0; q < kLuB; ++q)
    d[q] = (own && q < nbk) ? lu[static_cast<int64_t>(r0 + q) * n + r] : 0.0;
  if constexpr (!kUpper) {
#pragma unroll
    for (int q = 0; q < kLuB; ++q) {
      const double xq = __shfl(v, q);
      if (q < nbk && lane > q) v -= d[q] * xq;
    }
  } else {
#pragma unroll
    for (int q = kLuB - 1; q >= 0; --q) {
      if (q < nbk) {
        if (lane == q) v = v / d[q];
        const double xq = __shfl(v, q);
        if (lane < q) v -= d[q] * xq;
      }
    }
  }
  if (own) x[r] = v;
  __threadfence();
  if (lane == 0) __hip_atomic_store(flag + ci, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

// builds h->ap_* once; leaves ap_state = -1 if some row of A P has more
// distinct coarse columns than the per-row table holds
static void build_ap(Handle* h) {
  if (h->ap_state != 0) return;
  const int n = h->n;
  Allocator* al = &h->alloc;
  DBuf<int> err(al, 1);
  HIPX(hipMemsetAsync(err, 0, sizeof(int), h->stream));
  DBuf<int64_t> cnt(al, static_cast<size_t>(n) + 1);
  HIPX(hipMemsetAsync(cnt.get() + n, 0, sizeof(int64_t), h->stream));
  const unsigned g = static_cast<unsigned>((n + kApWaves - 1) / kApWaves);
  LAUNCH(h, "ap_count", k_ap<false>, g, 64 * kApWaves, 0, n, h->rp.get(), h->ci.get(),
         h->val.get(), h->p_rp.get(), h->p_ci.get(), h->p_val.get(), cnt.get(), nullptr, nullptr,
         err.get());
  int e = 0;
  HIPX(hipMemcpyAsync(&e, err.get(), sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  if (e != 0) {
    h->ap_state = -1;
    return;
  }
  h->ap_rp.reset(al, static_cast<size_t>(n) + 1);
  exclusive_scan_i64(h, cnt.get(), h->ap_rp.get(), n + 1);
  int64_t nnz = 0;
  HIPX(hipMemcpyAsync(&nnz, h->ap_rp.get() + n, sizeof(int64_t), hipMemcpyDeviceToHost,
                      h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  h->ap_ci.reset(al, std::max<int64_t>(nnz, 1));
  h->ap_val.reset(al, std::max<int64_t>(nnz, 1));
  LAUNCH(h, "ap_fill", k_ap<true>, g, 64 * kApWaves, 0, n, h->rp.get(), h->ci.get(),
         h->val.get(), h->p_rp.get(), h->p_ci.get(), h->p_val.get(), h->ap_rp.get(),
         h->ap_ci.get(), h->ap_val.get(), err.get());
  h->ap_state = 1;
}

void build_coarse_operator(Handle* h, const int* R_rp, const int* R_ci, const double* R_val,
                           int rows, double* out) {
  const int nc = h->nc;
  const int jt = std::min(nc, 4096);
  build_ap(h);
  if (h->ap_state == 1) {
    // all rows: one pass with hashed columns (the output zeroed first); rows
    // with too many columns for the table (none in the workloads here) are
    // redone by the tiled form, which also serves a build of fewer rows (it
    // writes only those)
    int herr = 1;
    if (rows == nc) {
      DBuf<int> err(&h->alloc, 1);
      HIPX(hipMemsetAsync(err, 0, sizeof(int), h->stream));
      HIPX(hipMemsetAsync(out, 0, static_cast<size_t>(nc) * nc * sizeof(double), h->stream));
      LAUNCH(h, "rap", k_rap_hash, rows, 64 * kRapWaves, 0, nc, R_rp, R_ci, R_val,
             h->ap_rp.get(), h->ap_ci.get(), h->ap_val.get(), out, err.get());
      HIPX(hipMemcpyAsync(&herr, err.get(), sizeof(int), hipMemcpyDeviceToHost, h->stream));
      HIPX(hipStreamSynchronize(h->stream));
    }
    if (herr) {
      const size_t lds = static_cast<size_t>(kRapWaves) * jt * sizeof(double);
      allow_lds(reinterpret_cast<const void*>(&k_rap_ap), lds);
      LAUNCH(h, "rap", k_rap_ap, rows, 64 * kRapWaves, lds, nc, R_rp, R_ci, R_val,
             h->ap_rp.get(), h->ap_ci.get(), h->ap_val.get(), out, jt);
    }
  } else {  // rows of A P too wide for the table: the direct triple product
    LAUNCH(h, "rap", k_rap, rows, 64, jt * sizeof(double), nc, R_rp, R_ci, R_val, h->rp.get(),
           h->ci.get(), h->val.get(), h->p_rp.get(), h->p_ci.get(), h->p_val.get(), out, jt);
  }
}

// LU with partial pivoting of `a` in place (P A = L U); perm (device, n):
// row i of P A is row perm[i] of A
void lu_factor(Handle* h, double* a, int n, int* perm_out) {
  DBuf<int> ipiv(&h->alloc, n), info(&h->alloc, 1);
  HIPX(hipMemsetAsync(info, 0, sizeof(int), h->stream));
  // panels of at most 4 * 512 rows live in registers (16 columns), larger
  // ones are factored in place (32 columns)
  auto width = [&](int k0) {
    const int m = n - k0;
    return m <= 4 * kRegThreads ? std::min(kRegNb, m) : std::min(kNb, m);
  };
  // a register panel can take in the update by a previous panel of at most
  // kRegNb columns (kpn > 0); a panel of k_panel cannot
  auto fusable = [&](int k0, int kpn) { return n - k0 <= 4 * kRegThreads && kpn <= kRegNb; };
  auto panel = [&](int k0, int nb, int kpn) {
    const int m = n - k0;
    if (m > 4 * kRegThreads)
      LAUNCH(h, "lu_panel", k_panel, 1, 1024, 0, a, n, k0, nb, ipiv.get(), info.get());
    else if (m > 2 * kRegThreads)
      LAUNCH(h, "lu_panel", k_panel_reg<4>, 1, kRegThreads, 0, a, n, k0, nb, ipiv.get(),
             info.get(), kpn);
    else if (m > kRegThreads)
      LAUNCH(h, "lu_panel", k_panel_reg<2>, 1, kRegThreads, 0, a, n, k0, nb, ipiv.get(),
             info.get(), kpn);
    else
      LAUNCH(h, "lu_panel", k_panel_reg<1>, 1, kRegThreads, 0, a, n, k0, nb, ipiv.get(),
             info.get(), kpn);
  };
  auto swap_trsm = [&](hipStream_t st, int k0, int nb, int lo1, int n1, int lo2, int n2) {
    if (n1 + n2 > 0)
      LAUNCH_ON(h, st, "lu_trsm", k_swap_trsm, blocks_for(n1 + n2, 64), 64, 0, a, n, k0, nb,
                ipiv.get(), lo1, n1, lo2, n2);
  };
  auto col = [&](int c) { return a + static_cast<int64_t>(c) * n; };
  // Look-ahead: after panel k a side stream applies step k (interchanges,
  // triangular solve, trailing update) to every column except the next
  // panel's, while the main stream brings the next panel's columns up to
  // date (inside its panel kernel where it can, else by the same two
  // launches) and factors it.  The two streams touch disjoint columns; the
  // main stream waits for the side stream's previous step before the next
  // panel (those columns took that step's update there), and the side
  // stream waits for each panel.
  Fork fork(h);
  fork.next();  // the main stream
  const hipStream_t side = fork.next();
  hipEvent_t ev_panel = h->aux.step[0], ev_rest = h->aux.step[1];
  int k0 = 0, nb = width(0);
  panel(k0, nb, 0);
  while (true) {
    const int c0 = k0 + nb;
    const int nb2 = c0 < n ? width(c0) : 0, c1 = c0 + nb2;
    HIPX(hipEventRecord(ev_panel, h->stream));
    HIPX(hipStreamWaitEvent(side, ev_panel, 0));
    swap_trsm(side, k0, nb, 0, k0, c1, n - c1);
    gemm_sub(h, n - c0, n - c1, nb, col(k0) + c0, col(c1) + k0, col(c1) + c0, n, side);
    if (k0 > 0) HIPX(hipStreamWaitEvent(h->stream, ev_rest, 0));
    HIPX(hipEventRecord(ev_rest, side));
    if (c0 >= n) break;
    const bool fuse = fusable(c0, nb);
    if (!fuse) {
      swap_trsm(h->stream, k0, nb, c0, nb2, 0, 0);
      gemm_sub(h, n - c0, nb2, nb, col(k0) + c0, col(c0) + k0, col(c0) + c0, n);
    }
    panel(c0, nb2, fuse ? nb : 0);
    k0 = c0;
    nb = nb2;
  }
  fork.join();
  int hinfo = 0;
  std::vector<int> hp(n);
  HIPX(hipMemcpyAsync(&hinfo, info.get(), sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPX(hipMemcpyAsync(hp.data(), ipiv.get(), n * sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  FAMS_REQUIRE(hinfo == 0, FAMS_ERR_SINGULAR_COARSE, "zero pivot in the coarse LU");
  std::vector<int> perm(n);
  for (int r = 0; r < n; ++r) perm[r] = r;
  for (int j = 0; j < n; ++j) std::swap(perm[j], perm[hp[j]]);
  HIPX(hipMemcpyAsync(perm_out, perm.data(), n * sizeof(int), hipMemcpyHostToDevice, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
}

// LU of `a` (n x n, overwritten) and inv = A^{-1} = U^{-1} L^{-1} P
void lu_inverse(Handle* h, double* a, double* inv, int n) {
  DBuf<int> dperm(&h->alloc, n);
  lu_factor(h, a, n, dperm.get());
  LAUNCH(h, "perm_identity", k_perm_identity, blocks_for(static_cast<int64_t>(n) * n, 256), 256, 0,
         n, dperm.get(), inv);
  for (int k0 = 0; k0 < n; k0 += kNb) {  // L Y = P
    int nb = std::min(kNb, n - k0);
    LAUNCH(h, "inv_trsm_l", k_trsm_lower_unit, blocks_for(n, 64), 64, 0, a, n, k0, nb, inv, 0, n);
    int r0 = k0 + nb;
    if (r0 < n)
      gemm_sub(h, n - r0, n, nb, a + static_cast<int64_t>(k0) * n + r0, inv + k0, inv + r0, n);
  }
  for (int k0 = ((n - 1) / kNb) * kNb; k0 >= 0; k0 -= kNb) {  // U X = Y
    int nb = std::min(kNb, n - k0);
    LAUNCH(h, "inv_trsm_u", k_trsm_upper, blocks_for(n, 64), 64, 0, a, n, k0, nb, inv, 0, n);
    if (k0 > 0) gemm_sub(h, k0, n, nb, a + static_cast<int64_t>(k0) * n, inv + k0, inv, n);
  }
}

// inv = A^{-1} by blocked Gauss-Jordan without pivoting; false (inv
// undefined) if a pivot is not positive, i.e. A is not SPD
namespace {

// the 32-wide Gauss-Jordan steps on a contiguous n x n matrix (in place)
void gje_inner(Handle* h, double* a, int n, int* info) {
  for (int k0 = 0; k0 < n; k0 += kNb) {
    const int nb = std::min(kNb, n - k0);
    LAUNCH(h, "gje_block", k_gje_block, 1, 1024, 0, a, n, k0, nb, info);
    if (n > nb) LAUNCH(h, "gje_col", k_gje_col, blocks_for(n - nb, 8), 256, 0, a, n, k0, nb);
    gemm_mfma(h, n, n, nb, 1.0, a + static_cast<int64_t>(k0) * n, n, a + k0, n, a, n, k0,
              k0 + nb);
    if (n > nb) LAUNCH(h, "gje_row", k_gje_row, blocks_for(n - nb, 8), 256, 0, a, n, k0, nb);
  }
}

// D (nb x nb, leading dimension nb) <- a[k0:k0+nb, k0:k0+nb]
__global__ void k_block_get(const double* a, int n, int k0, int nb, double* D) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= static_cast<int64_t>(nb) * nb) return;
  const int i = static_cast<int>(e % nb), c = static_cast<int>(e / nb);
  D[e] = a[static_cast<int64_t>(k0 + c) * n + k0 + i];
}

// column block and diagonal block back into a: a[r, k0 + c] = C1[r, c] for r
// outside the block, D[r - k0, c] inside it
__global__ void k_block_put_cols(double* a, int n, int k0, int nb, const double* C1,
                                 const double* D) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= static_cast<int64_t>(n) * nb) return;
  const int r = static_cast<int>(e % n), c = static_cast<int>(e / n);
  a[static_cast<int64_t>(k0 + c) * n + r] =
      (r >= k0 && r < k0 + nb) ? D[static_cast<int64_t>(c) * nb + (r - k0)] : C1[e];
}

// row block back into a: a[k0 + i, c] = R1[i, c] for columns c outside the block
__global__ void k_block_put_rows(double* a, int n, int k0, int nb, const double* R1) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= static_cast<int64_t>(n) * nb) return;
  const int i = static_cast<int>(e % nb), c = static_cast<int>(e / nb);
  if (c < k0 || c >= k0 + nb) a[static_cast<int64_t>(c) * n + k0 + i] = R1[e];
}

}  // namespace

// In-place Gauss-Jordan inverse in blocks of kOb = 1024 (no pivoting; SPD
// A_c).  Block step with D the diagonal block, B its row block, C its column
// block and E the rest: D <- D^{-1} (by the 32-wide steps above), C <- -C
// D^{-1}, E <- E + C B (old B), B <- D^{-1} B.  The three products are FP64
// MFMA GEMMs of inner dimension 1024, so the update of E (2 n^2 1024 flops
// per step, n/1024 steps) reads and writes E once per 1024 columns: the E
// traffic of a step is then small against its arithmetic (measured on an
// n = 17810 coarse system: 454 ms of GEMM time with 256-wide blocks, 363 ms
// with 512, 331 ms with 1024).
constexpr int kOb = 1024;

bool spd_inverse(Handle* h, const double* a, double* inv, int n) {
  DBuf<int> info(&h->alloc, 1);
  HIPX(hipMemsetAsync(info, 0, sizeof(int), h->stream));
  HIPX(hipMemcpyAsync(inv, a, sizeof(double) * n * n, hipMemcpyDeviceToDevice, h->stream));
  if (n <= kOb) {
    gje_inner(h, inv, n, info.get());
  } else {
    DBuf<double> D(&h->alloc, static_cast<size_t>(kOb) * kOb);
    DBuf<double> C1(&h->alloc, static_cast<size_t>(n) * kOb);
    DBuf<double> R1(&h->alloc, static_cast<size_t>(n) * kOb);
    for (int k0 = 0; k0 < n; k0 += kOb) {
      const int nb = std::min(kOb, n - k0);
      const int64_t nbb = static_cast<int64_t>(nb) * nb, nnb = static_cast<int64_t>(n) * nb;
      LAUNCH(h, "gje_get", k_block_get, blocks_for(nbb, 256), 256, 0, inv, n, k0, nb, D.get());
      gje_inner(h, D, nb, info.get());
      // C1 = -C D^{-1} (rows inside the block are not used)
      gemm_mfma(h, n, nb, nb, -1.0, inv + static_cast<int64_t>(k0) * n, n, D, nb, C1, n, 0, 0,
                nullptr, true);
      // E += C1 B
      gemm_mfma(h, n, n, nb, 1.0, C1, n, inv + k0, n, inv, n, k0, k0 + nb);
      // R1 = D^{-1} B (columns inside the block are not used)
      gemm_mfma(h, nb, n, nb, 1.0, D, nb, inv + k0, n, R1, nb, 0, 0, nullptr, true);
      LAUNCH(h, "gje_put", k_block_put_rows, blocks_for(nnb, 256), 256, 0, inv, n, k0, nb,
             R1.get());
      LAUNCH(h, "gje_put", k_block_put_cols, blocks_for(nnb, 256), 256, 0, inv, n, k0, nb,
             C1.get(), D.get());
    }
  }
  int hinfo = 0;
  HIPX(hipMemcpyAsync(&hinfo, info.get(), sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  return hinfo == 0;
}

int lu_solve_limit() { return kLuSolveMax; }

void dense_gemm_add(Handle* h, int m, int p, int k, double alpha, const double* A, int lda,
                    const double* B, int ldb, double* C, int ldc) {
  gemm_mfma(h, m, p, k, alpha, A, lda, B, ldb, C, ldc);
}

// x = A^{-1} b from lu_factor's output (x and b may alias)
void lu_solve(Handle* h, const double* lu, const int* perm, int n, const double* b, double* x) {
  FAMS_REQUIRE(n <= kLuSolveMax, FAMS_ERR_CAPACITY, "coarse system too large for the LU solve");
  const int nch = (n + kLuB - 1) / kLuB;
  if (h->lu_flag_n < 2 * nch) {
    h->lu_flags.reset(&h->alloc, 2 * nch);
    HIPX(hipMemsetAsync(h->lu_flags, 0, 2 * nch * sizeof(int), h->stream));
    h->lu_flag_n = 2 * nch;
    h->lu_epoch = 0;
  }
  if (!h->lu_err.get()) {   // error word, two tickets, long waits
    h->lu_err.reset(&h->alloc, 4);
    HIPX(hipMemsetAsync(h->lu_err, 0, 4 * sizeof(int), h->stream));
  }
  HIPX(hipMemsetAsync(h->lu_err, 0, 3 * sizeof(int), h->stream));
  const int epoch = ++h->lu_epoch;
  const unsigned long long limit = wait_limit(h);
  DBuf<double> w1(&h->alloc, n), w2(&h->alloc, n);
  LAUNCH(h, "lu_solve", k_gather_perm, blocks_for(n, 256), 256, 0, n, perm, b, w1.get());
  LAUNCH(h, "lu_solve", k_lu_df<false>, nch, 64, 0, n, lu, static_cast<const double*>(w1.get()),
         w2.get(), h->lu_flags.get(), epoch, h->lu_err.get(), h->lu_err.get() + 1, limit);
  LAUNCH(h, "lu_solve", k_lu_df<true>, nch, 64, 0, n, lu, static_cast<const double*>(w2.get()), x,
         h->lu_flags.get() + nch, epoch, h->lu_err.get(), h->lu_err.get() + 2, limit);
  int e[4] = {};
  HIPX(hipMemcpyAsync(e, h->lu_err.get(), sizeof(e), hipMemcpyDeviceToHost, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  h->info.long_waits += e[3];
  HIPX(hipMemsetAsync(h->lu_err.get() + 3, 0, sizeof(int), h->stream));
  FAMS_REQUIRE(e[0] == 0, FAMS_ERR_DEVICE, "LU solve: a dependency wait exceeded its bound");
}

// part: [ceil(nc / 64) * nc] partial sums
void coarse_apply(Handle* h, const double* inv, int nc, const double* x, double* y,
                  double* part) {
  static_assert(kGemvChunk == 64, "partial buffer is sized for 64-column chunks");
  int nch = (nc + kGemvChunk - 1) / kGemvChunk;
  dim3 grid(blocks_for(nc, 256), nch);
  LAUNCH(h, "coarse_gemv", k_gemv_part, grid, 256, 0, nc, inv, x, part);
  LAUNCH(h, "coarse_gemv_red", k_gemv_reduce, blocks_for(nc, 256), 256, 0, nc, nch, part, y);
}

}  // namespace fams
