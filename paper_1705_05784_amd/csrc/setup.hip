// Setup, part 1: the F-AMS prolongation P and restriction R = P^T on the GPU.
//
// One rule covers the four coupling strategies of App. A (Decoupled, Frac,
// Rock, Coupled-AMS): every cell has a rank rho (its wirebasket class
// I=0 < F=1 < E=2 < V=3, lifted by 4 for the medium solved first in Frac- and
// Rock-AMS); in a non-vertex row a coupling is
//   lumped  when cut (cross-media in Decoupled-AMS, or between unmerged
//           same-class blocks in Coupled-AMS) or when rho(j) < rho(i) -- the
//           localisation assumption, with the entry moved to the diagonal
//           (the over/underlined blocks of App. A);
//   RHS     when rho(j) > rho(i): -A_ij P_j, higher-rank rows of P acting as
//           boundary data (App. A.1, last paragraph);
//   kept    when rho(j) = rho(i) and not cut.
// Local blocks = connected components of the kept couplings (dual edges,
// faces, interiors; merged across media in Coupled-AMS).  Blocks are solved
// level by level from the highest rank down, each by one workgroup with a
// banded LDL^T factorisation (the local matrices are symmetric M-matrices),
// many right-hand sides at once -- one per coarse column the block touches.
//
// Determinism: every ordering is fixed (stable sorts, per-thread sequential
// sums in CSR order), so repeated setups are bitwise identical.
#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <numeric>
#include <type_traits>

#include "band.hpp"
#include "order.hpp"
#include "internal.hpp"

namespace fams {
namespace {

enum : int8_t { C_NONE = 0, C_KEPT = 1, C_LUMPED = 2, C_RHS = 3 };

constexpr int kThreads = 256;
constexpr int kBigBlockThreads = 512;  // blocks whose band lives in global memory
constexpr int kMaxCols = 2048;      // coarse columns per block (RHS count)

enum ErrBits : int {
  E_VERTEX_RANGE = 1, E_VERTEX_CLASS = 2, E_VERTEX_DUP = 4, E_V_NOT_LISTED = 8,
  E_CLASS_RANGE = 16, E_FRAC_INTERIOR = 32, E_PRIMAL_RANGE = 64,
  E_NO_HIGHER = 128, E_PIVOT = 256, E_SOURCES = 512, E_COLS = 2048, E_WELL_CLASS = 4096,
};

// rho(i): the wirebasket class lifted by 4 in the medium solved first (Frac-
// AMS: fractures, App. A.2; Rock-AMS: the matrix, App. A.3); a well ranks
// above every cell of both media, so its perforated cells take it as
// Dirichlet data in all four strategies (the beta term of the skeleton
// equation, Sec. 3.1)
__device__ __forceinline__ int rank_of(int wb, int i, int nm, int nwb, int variant) {
  const int med = medium_of(i, nm, nwb);
  if (med == 2) return 8;
  if (variant == FAMS_FRAC) return wb + (med == 1 ? 4 : 0);
  if (variant == FAMS_ROCK) return wb + (med == 1 ? 0 : 4);
  return wb;
}

__global__ void k_validate(int n, int nm, int nwb, int nc, const int8_t* wb, const int* primal,
                           const int64_t* vertex, int* coarse_of, int8_t* rho, int variant,
                           int* err) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nc) {
    int64_t v = vertex[i];
    if (v < 0 || v >= n) {
      atomicOr(err, E_VERTEX_RANGE);
    } else {
      if (wb[v] != 3) atomicOr(err, E_VERTEX_CLASS);
      if (atomicCAS(&coarse_of[v], -1, i) != -1) atomicOr(err, E_VERTEX_DUP);
    }
  }
  if (i < n) {
    int w = wb[i];
    if (w < 0 || w > 3) atomicOr(err, E_CLASS_RANGE);
    if (i >= nm && w == 0) atomicOr(err, E_FRAC_INTERIOR);
    if (i >= nwb && w != 3) atomicOr(err, E_WELL_CLASS);
    if (primal[i] < 0 || primal[i] >= nc) atomicOr(err, E_PRIMAL_RANGE);
    rho[i] = static_cast<int8_t>(rank_of(w, i, nm, nwb, variant));
  }
}

__global__ void k_check_vertices(int n, const int8_t* wb, const int* coarse_of, int* err) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && wb[i] == 3 && coarse_of[i] < 0) atomicOr(err, E_V_NOT_LISTED);
}

// Class of every stored entry.  `mode` = the variant whose rule is applied;
// `group` (Coupled only) = merged block label of each cell.
// Couplings with a well are never cut (wells are neither medium).
__global__ void k_classify(int n, int nm, int nwb, const int* rp, const int* ci, const int8_t* wb,
                           const int8_t* rho, int mode, const int* group, int8_t* ecls) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool vi = wb[i] == 3;
  const int mi = medium_of(i, nm, nwb);
  int ri = rho[i];
  for (int p = rp[i]; p < rp[i + 1]; ++p) {
    int j = ci[p];
    int8_t c = C_NONE;
    if (!vi && j != i) {
      const int mj = medium_of(j, nm, nwb);
      bool cross = mi != mj && mi < 2 && mj < 2;
      bool cut = false;
      if (mode == FAMS_DECOUPLED) cut = cross;
      else if (mode == FAMS_COUPLED) cut = cross && wb[i] == wb[j] && group[i] != group[j];
      int rj = rho[j];
      if (cut || rj < ri) c = C_LUMPED;
      else if (rj > ri) c = C_RHS;
      else c = C_KEPT;
    }
    ecls[p] = c;
  }
}

__global__ void k_label_init(int n, const int8_t* wb, int* label) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) label[i] = wb[i] == 3 ? -1 : i;
}

// hook: pull the smallest label over kept neighbours, and hook the old root
__global__ void k_label_hook(int n, const int* rp, const int* ci, const int8_t* ecls, int* label,
                             int* changed) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int li = label[i];
  if (li < 0) return;
  int m = li;
  for (int p = rp[i]; p < rp[i + 1]; ++p)
    if (ecls[p] == C_KEPT) m = min(m, label[ci[p]]);
  if (m < li) {
    atomicMin(&label[li], m);
    atomicMin(&label[i], m);
    *changed = 1;
  }
}

// compress: follow the label chain (strictly decreasing) to its root
__global__ void k_label_jump(int n, int* label) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int l = label[i];
  if (l < 0) return;
  while (true) {
    int nl = label[l];
    if (nl == l) break;
    l = nl;
  }
  label[i] = l;
}

// Coupled-AMS: cross-media couplings between non-vertex cells of one class, i < j
__global__ void k_cross_count(int n, int nm, const int* rp, const int* ci, const int8_t* wb,
                              int* cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = 0;
  if (wb[i] != 3) {
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      int j = ci[p];
      if (j > i && wb[j] == wb[i] && ((i >= nm) != (j >= nm))) ++c;
    }
  }
  cnt[i] = c;
}

__global__ void k_cross_fill(int n, int nm, const int* rp, const int* ci, const int8_t* wb,
                             const int* off, int* pairs) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || wb[i] == 3) return;
  int o = off[i];
  for (int p = rp[i]; p < rp[i + 1]; ++p) {
    int j = ci[p];
    if (j > i && wb[j] == wb[i] && ((i >= nm) != (j >= nm))) {
      pairs[2 * o] = i;
      pairs[2 * o + 1] = j;
      ++o;
    }
  }
}

__global__ void k_root_flags(int n, const int* label, int* flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = label[i] == i ? 1 : 0;
}

__global__ void k_root_keys(int n, const int* label, const int8_t* rho, const int* pos, int* keys,
                            int* vals) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && label[i] == i) {
    keys[pos[i]] = 7 - rho[i];
    vals[pos[i]] = i;
  }
}

__global__ void k_comp_index(int ncomp, const int* root_sorted, int* croot) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < ncomp) croot[root_sorted[k]] = k;
}

__global__ void k_comp_of(int n, const int* label, const int* croot, int* comp_of, int* flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int l = label[i];
  comp_of[i] = l < 0 ? -1 : croot[l];
  flag[i] = l < 0 ? 0 : 1;
}

__global__ void k_cell_keys(int n, const int* comp_of, const int* pos, int* keys, int* vals) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && comp_of[i] >= 0) {
    keys[pos[i]] = comp_of[i];
    vals[pos[i]] = i;
  }
}

__global__ void k_comp_ptr(int m, int ncomp, const int* key_sorted, const int* cells,
                           int* comp_ptr, int* local_idx) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m) return;
  int k = key_sorted[t];
  if (t == 0 || key_sorted[t - 1] != k) comp_ptr[k] = t;
  if (t == m - 1) comp_ptr[ncomp] = m;
  (void)cells;
}

__global__ void k_local_idx(int m, const int* key_sorted, const int* cells, const int* comp_ptr,
                            int* local_idx) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < m) local_idx[cells[t]] = t - comp_ptr[key_sorted[t]];
}

// kept couplings of a basis block
struct KeptEdge {
  const int8_t* ecls;
  __device__ bool operator()(int p, int, int) const { return ecls[p] == C_KEPT; }
};

__device__ __forceinline__ int bsearch_i32(const int* a, int n, int key) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Insert-if-absent into an open-addressing LDS hash set (EMPTY = INT_MIN);
// returns false when the table is full.
constexpr int kEmpty = INT_MIN;
__device__ __forceinline__ bool hset_insert(int* tab, int mask, int key, int* count) {
  unsigned h = (static_cast<unsigned>(key) * 2654435761u) & static_cast<unsigned>(mask);
  for (int probe = 0; probe <= mask; ++probe) {
    int prev = atomicCAS(&tab[h], kEmpty, key);
    if (prev == kEmpty) {
      atomicAdd(count, 1);
      return true;
    }
    if (prev == key) return true;
    h = (h + 1) & static_cast<unsigned>(mask);
  }
  return false;
}

// move the set's keys into out[0..count) and sort them ascending
__device__ void hset_collect_sorted(const int* tab, int size, int* out, int count, int* cursor) {
  if (threadIdx.x == 0) *cursor = 0;
  __syncthreads();
  for (int t = threadIdx.x; t < size; t += blockDim.x)
    if (tab[t] != kEmpty) out[atomicAdd(cursor, 1)] = tab[t];
  __syncthreads();
  block_bitonic_sort(out, count);
}

constexpr int kSrcSlots = 2048;   // hash slots for distinct higher-rank neighbour blocks
constexpr int kColSlots = 4096;   // hash slots for distinct coarse columns

// Symbolic pass of one rank level: the coarse columns each block's
// right-hand side touches (union over its higher-rank neighbours' columns),
// and the block's bandwidth in its local order.
__global__ void __launch_bounds__(kThreads)
k_colset(int c0, const int* comp_ptr, const int* cells, const int* rp, const int* ci,
         const int8_t* ecls, const int8_t* wb, const int* coarse_of, const int* comp_of,
         const int* local_idx, const int64_t* col_ptr, const int* cols, int* tmp_cols,
         int* ncols_out, int* band_out, int* err, int* diag) {
  __shared__ int src_tab[kSrcSlots];
  __shared__ int src[kSrcSlots];
  __shared__ int col_tab[kColSlots];
  __shared__ int colv[kColSlots];
  __shared__ int s_nsrc, s_ncol, s_band, s_over, s_cur;
  int K = c0 + blockIdx.x;
  int beg = comp_ptr[K], n = comp_ptr[K + 1] - beg;
  for (int t = threadIdx.x; t < kSrcSlots; t += blockDim.x) src_tab[t] = kEmpty;
  for (int t = threadIdx.x; t < kColSlots; t += blockDim.x) col_tab[t] = kEmpty;
  if (threadIdx.x == 0) {
    s_nsrc = 0;
    s_ncol = 0;
    s_band = 0;
    s_over = 0;
  }
  __syncthreads();
  int bmax = 0;
  bool over = false;
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    int i = cells[beg + l];
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      int8_t c = ecls[p];
      int j = ci[p];
      if (c == C_KEPT) {
        bmax = max(bmax, abs(local_idx[j] - local_idx[i]));
      } else if (c == C_RHS) {
        int sk = wb[j] == 3 ? -(coarse_of[j] + 1) : comp_of[j];
        if (!hset_insert(src_tab, kSrcSlots - 1, sk, &s_nsrc)) over = true;
      }
    }
  }
  atomicMax(&s_band, bmax);
  if (over) atomicOr(&s_over, E_SOURCES);
  __syncthreads();
  const int nsrc = s_nsrc;
  if (s_over || nsrc > kSrcSlots / 2) {
    if (threadIdx.x == 0) {
      atomicOr(err, E_SOURCES);
      if (atomicCAS(&diag[0], -1, K) == -1) {
        diag[1] = nsrc;
        diag[2] = n;
      }
    }
    return;
  }
  hset_collect_sorted(src_tab, kSrcSlots, src, nsrc, &s_cur);
  over = false;
  for (int t = threadIdx.x; t < nsrc; t += blockDim.x) {
    int sk = src[t];
    if (sk < 0) {
      if (!hset_insert(col_tab, kColSlots - 1, -sk - 1, &s_ncol)) over = true;
    } else {
      for (int64_t q = col_ptr[sk]; q < col_ptr[sk + 1]; ++q)
        if (!hset_insert(col_tab, kColSlots - 1, cols[q], &s_ncol)) over = true;
    }
  }
  if (over) atomicOr(&s_over, E_COLS);
  __syncthreads();
  const int nu = s_ncol;
  if (s_over || nu > kMaxCols) {
    if (threadIdx.x == 0) {
      atomicOr(err, E_COLS);
      if (atomicCAS(&diag[0], -1, K) == -1) {
        diag[1] = nsrc;
        diag[2] = n;
        diag[3] = nu;
      }
    }
    return;
  }
  if (nu == 0 && threadIdx.x == 0) atomicOr(err, E_NO_HIGHER);
  hset_collect_sorted(col_tab, kColSlots, colv, nu, &s_cur);
  int* out = tmp_cols + static_cast<int64_t>(blockIdx.x) * kMaxCols;
  for (int t = threadIdx.x; t < nu; t += blockDim.x) out[t] = colv[t];
  if (threadIdx.x == 0) {
    ncols_out[K] = nu;
    band_out[K] = s_band;
  }
}

__global__ void k_colcopy(int c0, int ncomp_level, const int* tmp_cols, const int64_t* col_ptr,
                          int* cols) {
  int K = c0 + blockIdx.x;
  int64_t a = col_ptr[K], b = col_ptr[K + 1];
  const int* src = tmp_cols + static_cast<int64_t>(blockIdx.x) * kMaxCols;
  for (int64_t t = threadIdx.x; t < b - a; t += blockDim.x) cols[a + t] = src[t];
  (void)ncomp_level;
}

// Numeric pass of one rank level: assemble A'_KK (band) and B_K, factor
// A'_KK = L D L^T (L unit lower, stored unscaled as L*D), solve for all
// right-hand sides.  TS = storage type of the P value pool, TC = arithmetic
// type.  With TS == TC the solution overwrites B_K in the pool; otherwise it
// is computed in `xwork` and rounded into the pool.  `list` (optional)
// selects the blocks: block = list[blockIdx.x], else c0 + blockIdx.x.
template <class TS, class TC>
__global__ void __launch_bounds__(kBigBlockThreads)
k_local_solve(const int* list, int c0, const int* comp_ptr, const int* cells, const int* rp,
              const int* ci, const double* av, const int8_t* ecls, const int8_t* wb,
              const int* coarse_of, const int* comp_of, const int* local_idx,
              const int64_t* col_ptr, const int* cols, const int* ncols, const int* band,
              const int64_t* pval_off, TS* pvals, const int64_t* work_off, TC* band_glob,
              TC* xwork, int lds_elems, int* err, int* bad_block, unsigned long long* timing) {
  extern __shared__ double lds_d[];
  unsigned long long* tk = timing ? timing + kTickSlots * static_cast<int64_t>(blockIdx.x) : nullptr;
  if (tk && threadIdx.x == 0) tk[0] = wall_clock64();
  int slot = blockIdx.x;
  int K = list ? list[slot] : c0 + slot;
  int beg = comp_ptr[K], n = comp_ptr[K + 1] - beg;
  int b = band[K], w = b + 1;
  int nck = ncols[K];
  const int* kcols = cols + col_ptr[K];
  TC* X;
  if constexpr (std::is_same<TS, TC>::value) X = xwork ? xwork + work_off[2 * slot + 1] : pvals + pval_off[K];
  else X = xwork + work_off[2 * slot + 1];
  const int64_t bsz = static_cast<int64_t>(n) * w;
  const int mode = band_mode(n, b, lds_elems);
  TC* lds = reinterpret_cast<TC*>(lds_d);
  TC* G = band_glob + work_off[2 * slot];  // modes 1/2: band, then its columns
  TC* Lt = G + bsz;
  TC* B = mode == 0 ? lds + band_panel_elems(b) : G;

  for (int64_t t = threadIdx.x; t < bsz; t += blockDim.x) B[t] = TC(0);
  __syncthreads();
  for (int64_t t = threadIdx.x; t < static_cast<int64_t>(n) * nck; t += blockDim.x) X[t] = TC(0);
  __syncthreads();
  // assemble the band: one thread per block row, entries in CSR order
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    int i = cells[beg + l];
    double dg = 0.0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      int j = ci[p];
      int8_t c = ecls[p];
      if (j == i || c == C_LUMPED) {
        dg += av[p];
      } else if (c == C_KEPT) {
        int lj = local_idx[j];
        if (lj < l) B[static_cast<int64_t>(l) * w + b - (l - lj)] = static_cast<TC>(av[p]);
      }
    }
    B[static_cast<int64_t>(l) * w + b] = static_cast<TC>(dg);
  }
  // right-hand sides (-A_ij P_j for higher-rank j): one wave per block row,
  // lanes over the columns of P_j
  {
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, nwaves = blockDim.x / 64;
    for (int l = wave; l < n; l += nwaves) {
      int i = cells[beg + l];
      TC* xl = X + static_cast<int64_t>(l) * nck;
      for (int p = rp[i]; p < rp[i + 1]; ++p) {
        if (ecls[p] != C_RHS) continue;
        int j = ci[p];
        TC a = static_cast<TC>(av[p]);
        if (wb[j] == 3) {
          if (lane == 0) xl[bsearch_i32(kcols, nck, coarse_of[j])] -= a;
        } else {
          int cj = comp_of[j];
          int ncj = ncols[cj];
          const TS* src = pvals + pval_off[cj] + static_cast<int64_t>(local_idx[j]) * ncj;
          const int* cc = cols + col_ptr[cj];
          for (int t = lane; t < ncj; t += 64)
            xl[bsearch_i32(kcols, nck, cc[t])] -= a * static_cast<TC>(src[t]);
        }
        // the next entry may update the same positions from other lanes
        __threadfence_block();
      }
    }
  }
  __syncthreads();
  __syncthreads();
  if (tk && threadIdx.x == 0) {
    tk[1] = wall_clock64();
    tk[5] = (static_cast<unsigned long long>(n) << 32) | static_cast<unsigned>(b);
    tk[6] = (static_cast<unsigned long long>(nck) << 32) |
            static_cast<unsigned>(mode);
  }
  bool bad = band_factor<TC>(mode, G, Lt, n, b, lds, tk ? tk + 2 : nullptr);
  if (band_wave_class(b) != 0) {  // the substitution follows in k_local_subst
    if (mode == 0) band_export<TC>(lds + band_panel_elems(b), G, n, b);
  } else {
    band_substitute<TC, TC>(B, n, b, X, nck, lds);
    if (!std::is_same<TS, TC>::value || xwork) {
      TS* out = pvals + pval_off[K];
      for (int64_t t = threadIdx.x; t < static_cast<int64_t>(n) * nck; t += blockDim.x)
        out[t] = static_cast<TS>(X[t]);
    }
  }
  if (tk && threadIdx.x == 0) tk[4] = wall_clock64();
  if (bad && threadIdx.x == 0) {
    atomicOr(err, E_PIVOT);
    if (bad_block) bad_block[K] = 1;
  }
}

// Substitution of one rank level's local solves with the factors (band and
// Lt) that k_local_solve left in global memory: one wavefront per group of
// columns of one block, for the blocks of chunk-slot class M.
// groups[3 g ..] = (slot, first column, columns: 1 or 4).
template <class TS, class TC, int M>
__global__ void __launch_bounds__(64)
k_local_subst(const int* groups, const int* list, int c0, const int* comp_ptr, const int* ncols,
              const int* band, const int64_t* pval_off, TS* pvals, const int64_t* work_off,
              const TC* band_glob, TC* xwork, unsigned long long* timing) {
  unsigned long long t0 = timing ? wall_clock64() : 0;
  const int* gq = groups + 3 * static_cast<int64_t>(blockIdx.x);
  const int slot = gq[0], col = gq[1], nc = gq[2];
  const int K = list ? list[slot] : c0 + slot;
  const int n = comp_ptr[K + 1] - comp_ptr[K], b = band[K], nck = ncols[K];
  const TC* G = band_glob + work_off[2 * slot];
  const TC* Lt = G + static_cast<int64_t>(n) * (b + 1);
  TS* out = pvals + pval_off[K];
  TC* X;
  if constexpr (std::is_same<TS, TC>::value) X = xwork ? xwork + work_off[2 * slot + 1] : out;
  else X = xwork + work_off[2 * slot + 1];
  constexpr int J = sizeof(TC) == 4 ? 8 : 4;
  if (nc == 4) band_wave_columns<TC, TC, TS, M, 4, J>(G, Lt, 1, 0, n, b, X, nck, col, out);
  else band_wave_columns<TC, TC, TS, M, 1, J>(G, Lt, 1, 0, n, b, X, nck, col, out);
  if (timing && threadIdx.x == 0) {
    unsigned long long* tk = timing + 4 * static_cast<int64_t>(blockIdx.x);
    tk[0] = t0;
    tk[1] = wall_clock64();
    tk[2] = (static_cast<unsigned long long>(n) << 32) | static_cast<unsigned>(b);
    tk[3] = (static_cast<unsigned long long>(M) << 32) | static_cast<unsigned>(nc);
  }
}

// ---- local solves of a non-symmetric A (LU without pivoting) ---------------
// The same local problems as k_local_solve (A'_KK P_K = B_K) when A is not
// symmetric (a linearised compressible system): the full band of A'_KK
// (row l, columns l-b..l+b at B[l (2b+1) + b + (j - l)]) in global memory,
// factored in place into unit-lower L and upper U by right-looking
// elimination without pivoting (the local matrices are M-matrices), one
// elimination step per pair of barriers; then every thread substitutes whole
// columns of X (forward with L, backward with U), rows in order.  Plain, not
// blocked: the general-matrix path, not the symmetric one the benchmarks use.
template <class TS, class TC>
__global__ void __launch_bounds__(kThreads)
k_local_solve_lu(const int* list, const int* comp_ptr, const int* cells, const int* rp,
                 const int* ci, const double* av, const int8_t* ecls, const int8_t* wb,
                 const int* coarse_of, const int* comp_of, const int* local_idx,
                 const int64_t* col_ptr, const int* cols, const int* ncols, const int* band,
                 const int64_t* pval_off, TS* pvals, const int64_t* work_off, TC* band_glob,
                 TC* xwork, int* err, int* bad_block) {
  const int slot = blockIdx.x;
  const int K = list[slot];
  const int beg = comp_ptr[K], n = comp_ptr[K + 1] - beg;
  const int b = band[K], w = 2 * b + 1;
  const int nck = ncols[K];
  const int* kcols = cols + col_ptr[K];
  TC* X;
  if constexpr (std::is_same<TS, TC>::value) X = xwork ? xwork + work_off[2 * slot + 1] : pvals + pval_off[K];
  else X = xwork + work_off[2 * slot + 1];
  TC* B = band_glob + work_off[2 * slot];
  const int64_t bsz = static_cast<int64_t>(n) * w;
  for (int64_t t = threadIdx.x; t < bsz; t += blockDim.x) B[t] = TC(0);
  for (int64_t t = threadIdx.x; t < static_cast<int64_t>(n) * nck; t += blockDim.x) X[t] = TC(0);
  __syncthreads();
  // the band, both triangles: one thread per block row
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    const int i = cells[beg + l];
    double dg = 0.0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      const int j = ci[p];
      const int8_t c = ecls[p];
      if (j == i || c == C_LUMPED) dg += av[p];
      else if (c == C_KEPT) B[static_cast<int64_t>(l) * w + b + (local_idx[j] - l)] = static_cast<TC>(av[p]);
    }
    B[static_cast<int64_t>(l) * w + b] = static_cast<TC>(dg);
  }
  // right-hand sides -A_ij P_j of the higher-rank neighbours (as k_local_solve)
  {
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, nwaves = blockDim.x / 64;
    for (int l = wave; l < n; l += nwaves) {
      const int i = cells[beg + l];
      TC* xl = X + static_cast<int64_t>(l) * nck;
      for (int p = rp[i]; p < rp[i + 1]; ++p) {
        if (ecls[p] != C_RHS) continue;
        const int j = ci[p];
        const TC a = static_cast<TC>(av[p]);
        if (wb[j] == 3) {
          if (lane == 0) xl[bsearch_i32(kcols, nck, coarse_of[j])] -= a;
        } else {
          const int cj = comp_of[j];
          const int ncj = ncols[cj];
          const TS* src = pvals + pval_off[cj] + static_cast<int64_t>(local_idx[j]) * ncj;
          const int* cc = cols + col_ptr[cj];
          for (int t = lane; t < ncj; t += 64)
            xl[bsearch_i32(kcols, nck, cc[t])] -= a * static_cast<TC>(src[t]);
        }
        __threadfence_block();
      }
    }
  }
  __syncthreads();
  // LU: step k scales column k below the pivot, then updates the trailing
  // window of rows and columns k+1..k+b
  bool bad = false;
  for (int k = 0; k < n; ++k) {
    const int e = min(n - 1, k + b);
    const TC piv = B[static_cast<int64_t>(k) * w + b];
    if (!(piv > TC(0))) bad = true;
    for (int i = k + 1 + static_cast<int>(threadIdx.x); i <= e; i += blockDim.x)
      B[static_cast<int64_t>(i) * w + b + (k - i)] /= piv;
    __syncthreads();
    const int m = e - k;
    for (int t = threadIdx.x; t < m * m; t += blockDim.x) {
      const int i = k + 1 + t / m, j = k + 1 + t % m;
      B[static_cast<int64_t>(i) * w + b + (j - i)] -=
          B[static_cast<int64_t>(i) * w + b + (k - i)] * B[static_cast<int64_t>(k) * w + b + (j - k)];
    }
    __syncthreads();
  }
  // substitution, one thread per column
  for (int c = threadIdx.x; c < nck; c += blockDim.x) {
    for (int l = 0; l < n; ++l) {
      TC s = X[static_cast<int64_t>(l) * nck + c];
      for (int t = max(0, l - b); t < l; ++t)
        s -= B[static_cast<int64_t>(l) * w + b + (t - l)] * X[static_cast<int64_t>(t) * nck + c];
      X[static_cast<int64_t>(l) * nck + c] = s;
    }
    for (int l = n - 1; l >= 0; --l) {
      TC s = X[static_cast<int64_t>(l) * nck + c];
      for (int t = l + 1; t <= min(n - 1, l + b); ++t)
        s -= B[static_cast<int64_t>(l) * w + b + (t - l)] * X[static_cast<int64_t>(t) * nck + c];
      X[static_cast<int64_t>(l) * nck + c] = s / B[static_cast<int64_t>(l) * w + b];
    }
  }
  __syncthreads();
  if (!std::is_same<TS, TC>::value || xwork) {
    TS* out = pvals + pval_off[K];
    for (int64_t t = threadIdx.x; t < static_cast<int64_t>(n) * nck; t += blockDim.x)
      out[t] = static_cast<TS>(X[t]);
  }
  if (bad && threadIdx.x == 0) {
    atomicOr(err, E_PIVOT);
    if (bad_block) bad_block[K] = 1;
  }
}

// ---- P in CSR (with the optional truncation of Sec. 4.3) -------------------
template <class T>
__global__ void k_p_count(int n, const int8_t* wb, const int* comp_of, const int* local_idx,
                          const int* ncols, const int64_t* pval_off, const T* pvals, double alpha,
                          int* cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (wb[i] == 3) {
    cnt[i] = 1;
    return;
  }
  int K = comp_of[i];
  int nck = ncols[K];
  if (alpha <= 0.0) {
    cnt[i] = nck;
    return;
  }
  const T* v = pvals + pval_off[K] + static_cast<int64_t>(local_idx[i]) * nck;
  int c = 0;
  for (int t = 0; t < nck; ++t)
    if (fabs(static_cast<double>(v[t])) >= alpha) ++c;
  cnt[i] = c ? c : 1;
}

template <class T>
__global__ void k_p_fill(int n, const int8_t* wb, const int* coarse_of, const int* comp_of,
                         const int* local_idx, const int* ncols, const int64_t* col_ptr,
                         const int* cols, const int64_t* pval_off, const T* pvals, double alpha,
                         const int* p_rp, int* p_ci, double* p_val) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int o = p_rp[i];
  if (wb[i] == 3) {
    p_ci[o] = coarse_of[i];
    p_val[o] = 1.0;
    return;
  }
  int K = comp_of[i];
  int nck = ncols[K];
  const T* v = pvals + pval_off[K] + static_cast<int64_t>(local_idx[i]) * nck;
  const int* cc = cols + col_ptr[K];
  int kept = p_rp[i + 1] - o;
  if (alpha <= 0.0 || kept == nck) {
    bool all = true;
    if (alpha > 0.0)
      for (int t = 0; t < nck; ++t) all = all && fabs(static_cast<double>(v[t])) >= alpha;
    if (all) {
      for (int t = 0; t < nck; ++t) {
        p_ci[o + t] = cc[t];
        p_val[o + t] = static_cast<double>(v[t]);
      }
      return;
    }
  }
  double s0 = 0.0, s1 = 0.0;
  int nk = 0;
  for (int t = 0; t < nck; ++t) {
    double x = static_cast<double>(v[t]);
    s0 += x;
    if (fabs(x) >= alpha) {
      s1 += x;
      ++nk;
    }
  }
  if (nk == 0) {  // keep the largest entry (lowest column on ties)
    int best = 0;
    for (int t = 1; t < nck; ++t)
      if (fabs(static_cast<double>(v[t])) > fabs(static_cast<double>(v[best]))) best = t;
    double x = static_cast<double>(v[best]);
    p_ci[o] = cc[best];
    p_val[o] = s0 != 0.0 && x != 0.0 ? x * (s0 / x) : x;
    return;
  }
  double scale = s1 != 0.0 ? s0 / s1 : 1.0;
  for (int t = 0; t < nck; ++t) {
    double x = static_cast<double>(v[t]);
    if (fabs(x) >= alpha) {
      p_ci[o] = cc[t];
      p_val[o] = x * scale;
      ++o;
    }
  }
}

__global__ void k_entry_rows(int n, const int* rp, int* erow, int* iota) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int p = rp[i]; p < rp[i + 1]; ++p) {
    erow[p] = i;
    iota[p] = p;
  }
}

__global__ void k_r_fill(int64_t nnz, int nc, const int* key_sorted, const int* perm,
                         const int* erow, const double* p_val, int* r_rp, int* r_ci,
                         double* r_val) {
  int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  int e = perm[k];
  r_ci[k] = erow[e];
  r_val[k] = p_val[e];
  int J = key_sorted[k];
  int Jprev = k == 0 ? -1 : key_sorted[k - 1];
  for (int c = Jprev + 1; c <= J; ++c) r_rp[c] = static_cast<int>(k);
  if (k == nnz - 1)
    for (int c = J + 1; c <= nc; ++c) r_rp[c] = static_cast<int>(nnz);
}

__global__ void k_d2f(int64_t n, const double* a, float* b) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) b[i] = static_cast<float>(a[i]);
}

int bits_for(int64_t v) {
  int b = 1;
  while ((int64_t(1) << b) <= v) ++b;
  return b;
}

template <class T>
int64_t read1(Handle* h, const T* dev) {
  T v{};
  HIPX(hipMemcpyAsync(&v, dev, sizeof(T), hipMemcpyDeviceToHost, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  return static_cast<int64_t>(v);
}

std::string grid_error_text(int e) {
  std::string s = "grid:";
  if (e & E_VERTEX_RANGE) s += " vertex index out of range;";
  if (e & E_VERTEX_CLASS) s += " a listed vertex is not of class V;";
  if (e & E_VERTEX_DUP) s += " a cell listed twice as vertex;";
  if (e & E_V_NOT_LISTED) s += " a class-V cell missing from the vertex list;";
  if (e & E_CLASS_RANGE) s += " wirebasket class outside 0..3;";
  if (e & E_FRAC_INTERIOR) s += " fracture cell of class I;";
  if (e & E_WELL_CLASS) s += " a well is not of class V (every well is a coarse node);";
  if (e & E_PRIMAL_RANGE) s += " primal id out of range;";
  return s;
}

// connected components of the kept couplings (hook and compress)
void components(Handle* h, const int8_t* wb, const int8_t* ecls, int* label) {
  int n = h->n;
  unsigned g = blocks_for(n, kThreads);
  LAUNCH(h, "label_init", k_label_init, g, kThreads, 0, n, wb, label);
  DBuf<int> changed(&h->alloc, 1);
  for (int it = 0; it < 100000; ++it) {
    HIPX(hipMemsetAsync(changed, 0, sizeof(int), h->stream));
    LAUNCH(h, "label_hook", k_label_hook, g, kThreads, 0, n, h->rp.get(), h->ci.get(), ecls, label,
           changed.get());
    LAUNCH(h, "label_jump", k_label_jump, g, kThreads, 0, n, label);
    if (!read1(h, changed.get())) return;
  }
  throw Error(FAMS_ERR_DEVICE, "component labelling did not converge");
}

// Coupled-AMS merge of same-class blocks across media, in CSR order, under
// the merge cap (host union-find over the short list of cross couplings)
void coupled_groups(Handle* h, const int8_t* wb, const int* base, int* group) {
  int n = h->n, nm = h->nm;
  unsigned g = blocks_for(n, kThreads);
  DBuf<int> cnt(&h->alloc, n), off(&h->alloc, n);
  LAUNCH(h, "cross_count", k_cross_count, g, kThreads, 0, n, nm, h->rp.get(), h->ci.get(), wb,
         cnt.get());
  exclusive_scan_i32(h, cnt, off, n);
  int64_t m = read1(h, off.get() + n - 1) + read1(h, cnt.get() + n - 1);
  std::vector<int> hb(n), pairs(2 * m);
  if (m) {
    DBuf<int> dp(&h->alloc, 2 * m);
    LAUNCH(h, "cross_fill", k_cross_fill, g, kThreads, 0, n, nm, h->rp.get(), h->ci.get(), wb,
           off.get(), dp.get());
    HIPX(hipMemcpyAsync(pairs.data(), dp.get(), 2 * m * sizeof(int), hipMemcpyDeviceToHost,
                        h->stream));
  }
  HIPX(hipMemcpyAsync(hb.data(), base, n * sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  std::vector<int> parent(n), size(n, 0);
  std::iota(parent.begin(), parent.end(), 0);
  for (int i = 0; i < n; ++i)
    if (hb[i] >= 0) ++size[hb[i]];
  auto find = [&](int a) {
    while (parent[a] != a) {
      parent[a] = parent[parent[a]];
      a = parent[a];
    }
    return a;
  };
  for (int64_t e = 0; e < m; ++e) {
    int a = find(hb[pairs[2 * e]]), b = find(hb[pairs[2 * e + 1]]);
    if (a == b) continue;
    if (static_cast<int64_t>(size[a]) + size[b] <= h->merge_cap) {
      int lo = std::min(a, b), hi = std::max(a, b);
      parent[hi] = lo;
      size[lo] += size[hi];
    }
  }
  for (int i = 0; i < n; ++i) hb[i] = hb[i] >= 0 ? find(hb[i]) : -1;
  HIPX(hipMemcpyAsync(group, hb.data(), n * sizeof(int), hipMemcpyHostToDevice, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
}

// Launch the local solves of blocks `blocks` (all of one rank level).
template <class TS, class TC>
void local_solves(Handle* h, const std::vector<int>& blocks, bool use_list, const int* comp_ptr,
                  const int* cells, const int8_t* ecls, const int8_t* wb, const int* coarse_of,
                  const int* comp_of, const int* local_idx, const int64_t* col_ptr,
                  const int* cols, const int* ncols, const int* band, const int64_t* pval_off,
                  TS* pvals, const std::vector<int>& h_comp_ptr, const std::vector<int>& h_band,
                  const std::vector<int>& h_ncols, int* err, int* bad_block) {
  const int nb = static_cast<int>(blocks.size());
  if (nb == 0) return;
  (void)use_list;
  const bool separate_x = !std::is_same<TS, TC>::value;
  if (h->nonsym) {  // the general path: full band in global memory, LU in place
    std::vector<int64_t> off(2 * nb, 0);
    int64_t band_total = 0, x_total = 0;
    for (int k = 0; k < nb; ++k) {
      const int K = blocks[k];
      const int64_t nk = h_comp_ptr[K + 1] - h_comp_ptr[K];
      off[2 * k] = band_total;
      band_total += nk * (2 * h_band[K] + 1);
      off[2 * k + 1] = x_total;
      if (separate_x) x_total += nk * h_ncols[K];
      const double bw = h_band[K], nn = static_cast<double>(nk);
      h->info.local_flops += 2.0 * nn * bw * bw + 4.0 * nn * bw * h_ncols[K];
    }
    DBuf<int64_t> d_off(&h->alloc, 2 * nb);
    HIPX(hipMemcpyAsync(d_off, off.data(), 2 * nb * sizeof(int64_t), hipMemcpyHostToDevice,
                        h->stream));
    DBuf<int> d_list(&h->alloc, nb);
    HIPX(hipMemcpyAsync(d_list, blocks.data(), nb * sizeof(int), hipMemcpyHostToDevice,
                        h->stream));
    DBuf<TC> scratch(&h->alloc, std::max<int64_t>(band_total, 1));
    DBuf<TC> xw;
    if (separate_x) xw.reset(&h->alloc, std::max<int64_t>(x_total, 1));
    LAUNCH(h, "local_solve_lu", (k_local_solve_lu<TS, TC>), nb, kThreads, 0,
           static_cast<const int*>(d_list.get()), comp_ptr, cells, h->rp.get(), h->ci.get(),
           h->val.get(), ecls, wb, coarse_of, comp_of, local_idx, col_ptr, cols, ncols, band,
           pval_off, pvals, static_cast<const int64_t*>(d_off.get()), scratch.get(), xw.get(),
           err, bad_block);
    HIPX(hipStreamSynchronize(h->stream));  // scratch is freed on return
    return;
  }
  const int64_t lds_cap = lds_budget(h) / static_cast<int64_t>(sizeof(TC));
  // slots: the blocks whose band fits in LDS (in the given order), then the
  // others, longest first, which get a launch of their own with more waves
  std::vector<int> blk, big;
  for (int K : blocks) {
    const int nk = h_comp_ptr[K + 1] - h_comp_ptr[K];
    const int mode = band_mode(nk, h_band[K], lds_cap);
    FAMS_REQUIRE(mode >= 0, FAMS_ERR_CAPACITY, "local block bandwidth too large for LDS");
    (mode == 0 ? blk : big).push_back(K);
  }
  std::stable_sort(big.begin(), big.end(), [&](int a, int b) {
    return h_comp_ptr[a + 1] - h_comp_ptr[a] > h_comp_ptr[b + 1] - h_comp_ptr[b];
  });
  const int n_small = static_cast<int>(blk.size());
  blk.insert(blk.end(), big.begin(), big.end());
  std::vector<int64_t> off(2 * nb, 0);
  int64_t band_total = 0, x_total = 0, lds_small = 0, lds_big = 0;
  for (int k = 0; k < nb; ++k) {
    int K = blk[k];
    int64_t nk = h_comp_ptr[K + 1] - h_comp_ptr[K];
    const int mode = band_mode(static_cast<int>(nk), h_band[K], lds_cap);
    off[2 * k] = band_total;
    band_total += 2 * nk * (h_band[K] + 1);  // factor band and Lt in global memory
    int64_t& need = k < n_small ? lds_small : lds_big;
    need = std::max(need, band_lds_elems(mode, static_cast<int>(nk), h_band[K]));
    off[2 * k + 1] = x_total;
    if (separate_x) x_total += nk * h_ncols[K];
    {  // arithmetic of the band LDL^T (step k updates a triangle of
       // min(b, n-1-k) rows) and of the two sweeps for each column
      const double b = h_band[K], nn = static_cast<double>(nk), t = std::min(b, nn);
      const double fac = std::max(0.0, nn - b) * b * (b + 1.0) + (t - 1.0) * t * (t + 1.0) / 3.0;
      const double S = nn >= b ? nn * b - b * (b + 1.0) / 2.0 : nn * (nn - 1.0) / 2.0;
      const double sub = (4.0 * S + nn) * h_ncols[K];
      h->info.local_flops += fac;
      if (band_wave_class(h_band[K]) != 0) h->info.local_subst_flops += sub;
      else h->info.local_flops += sub;
    }
  }
  DBuf<int64_t> d_off(&h->alloc, 2 * nb);
  HIPX(hipMemcpyAsync(d_off, off.data(), 2 * nb * sizeof(int64_t), hipMemcpyHostToDevice,
                      h->stream));
  DBuf<int> d_list(&h->alloc, nb);
  HIPX(hipMemcpyAsync(d_list, blk.data(), nb * sizeof(int), hipMemcpyHostToDevice, h->stream));
  DBuf<TC> scratch(&h->alloc, std::max<int64_t>(band_total, 1));
  DBuf<TC> xw;
  if (separate_x) xw.reset(&h->alloc, std::max<int64_t>(x_total, 1));
  allow_lds(reinterpret_cast<const void*>(&k_local_solve<TS, TC>),
            std::max(lds_small, lds_big) * sizeof(TC));
  static const bool timing_on = std::getenv("FAMS_BLOCK_TIMING") != nullptr;
  DBuf<unsigned long long> timing;
  if (timing_on) {
    timing.reset(&h->alloc, kTickSlots * static_cast<size_t>(nb));
    HIPX(hipMemsetAsync(timing, 0, kTickSlots * nb * sizeof(unsigned long long), h->stream));
  }
  {
    Fork fork(h);
    for (int part = 0; part < 2; ++part) {  // slots [s0, s1)
      const int s0 = part ? n_small : 0, s1 = part ? nb : n_small;
      if (s1 == s0) continue;
      const int lds_elems = static_cast<int>(part ? lds_big : lds_small);
      hipStream_t st = fork.next();
      LAUNCH_ON(h, st, "local_solve", (k_local_solve<TS, TC>), s1 - s0,
                part ? kBigBlockThreads : kThreads, lds_elems * sizeof(TC),
                static_cast<const int*>(d_list.get() + s0), 0, comp_ptr, cells, h->rp.get(),
                h->ci.get(), h->val.get(), ecls, wb, coarse_of, comp_of, local_idx, col_ptr, cols,
                ncols, band, pval_off, pvals, d_off.get() + 2 * s0, scratch.get(), xw.get(),
                lds_elems, err, bad_block, timing_on ? timing.get() + kTickSlots * s0 : nullptr);
    }
    fork.join();
  }
  if (timing_on) {
    HIPX(hipStreamSynchronize(h->stream));
    if (n_small) print_block_timing(timing.get(), n_small, blocks[0]);
    if (nb > n_small)
      print_block_timing(timing.get() + kTickSlots * n_small, nb - n_small, blocks[0]);
  }
  // substitutions: groups of 4 columns, then single columns, per slot class
  // (classes on separate streams; within a class the longest blocks first)
  std::vector<int> order(nb);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return h_comp_ptr[blk[a] + 1] - h_comp_ptr[blk[a]] >
           h_comp_ptr[blk[b] + 1] - h_comp_ptr[blk[b]];
  });
  std::vector<int> groups;
  std::vector<std::pair<int, int>> cls;  // (class, groups in it)
  for (int m : {2, 3, 4, 5, 6, 7, 9}) {
    const size_t g0 = groups.size();
    for (int k : order) {
      const int K = blk[k];
      if (band_wave_class(h_band[K]) != m) continue;
      const int nck = h_ncols[K];
      for (int c = 0; c + 4 <= nck; c += 4) groups.insert(groups.end(), {k, c, 4});
      for (int c = nck - nck % 4; c < nck; ++c) groups.insert(groups.end(), {k, c, 1});
    }
    const int ng = static_cast<int>((groups.size() - g0) / 3);
    if (ng) cls.emplace_back(m, ng);
  }
  DBuf<int> d_groups(&h->alloc, std::max<size_t>(groups.size(), 1));
  if (!groups.empty())
    HIPX(hipMemcpyAsync(d_groups, groups.data(), groups.size() * sizeof(int),
                        hipMemcpyHostToDevice, h->stream));
  DBuf<unsigned long long> sub_timing;
  if (timing_on) sub_timing.reset(&h->alloc, 4 * std::max<size_t>(groups.size() / 3, 1));
  int64_t gofs = 0;
  Fork fork(h);
  for (auto [m, ng] : cls) {
    hipStream_t st = fork.next();
#define FAMS_SUBST(M)                                                                         \
  LAUNCH_ON(h, st, "local_subst", (k_local_subst<TS, TC, M>), ng, 64, 0,                      \
         static_cast<const int*>(d_groups.get() + 3 * gofs), static_cast<const int*>(d_list.get()), \
         blocks[0], comp_ptr, ncols, band, pval_off, pvals, static_cast<const int64_t*>(d_off.get()), \
         static_cast<const TC*>(scratch.get()), xw.get(),                                      \
         timing_on ? sub_timing.get() + 4 * gofs : nullptr)
    switch (m) {
      case 2: FAMS_SUBST(2); break;
      case 3: FAMS_SUBST(3); break;
      case 4: FAMS_SUBST(4); break;
      case 5: FAMS_SUBST(5); break;
      case 6: FAMS_SUBST(6); break;
      case 7: FAMS_SUBST(7); break;
      default: FAMS_SUBST(9); break;
    }
#undef FAMS_SUBST
    gofs += ng;
  }
  fork.join();
  HIPX(hipStreamSynchronize(h->stream));  // scratch is freed on return
  if (timing_on && !groups.empty()) {  // the launch span and its longest wavefronts
    const size_t ng = groups.size() / 3;
    std::vector<unsigned long long> t(4 * ng);
    HIPX(hipMemcpy(t.data(), sub_timing.get(), t.size() * sizeof(unsigned long long),
                   hipMemcpyDeviceToHost));
    unsigned long long lo = ~0ull, hi = 0;
    std::vector<std::pair<unsigned long long, size_t>> d(ng);
    for (size_t g = 0; g < ng; ++g) {
      lo = std::min(lo, t[4 * g]);
      hi = std::max(hi, t[4 * g + 1]);
      d[g] = {t[4 * g + 1] - t[4 * g], g};
    }
    std::sort(d.begin(), d.end(), [](auto& a, auto& b) { return a.first > b.first; });
    std::fprintf(stderr, "[subst from %d] %zu wavefronts, span %llu ticks\n", blocks[0], ng, hi - lo);
    for (size_t q = 0; q < std::min<size_t>(ng, 4); ++q) {
      const unsigned long long* r = &t[4 * d[q].second];
      std::fprintf(stderr, "   n %llu b %llu M %llu cols %llu : %llu ticks (start +%llu)\n",
                   r[2] >> 32, r[2] & 0xffffffffull, r[3] >> 32, r[3] & 0xffffffffull, d[q].first,
                   r[0] - lo);
    }
  }
}

}  // namespace

// FAMS_BLOCK_TIMING=1: per-block phase durations of one launch to stderr
// (wall-clock ticks of the device's constant-rate counter): the launch's
// span, the summed phases per storage mode and the slowest blocks.
void print_block_timing(const unsigned long long* dev, int nb, int first) {
  std::vector<unsigned long long> t(kTickSlots * static_cast<size_t>(nb));
  HIPX(hipMemcpy(t.data(), dev, t.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
  double sum[3][5] = {};
  int cnt[3] = {0, 0, 0};
  unsigned long long t_first = ~0ull, t_last = 0;
  std::vector<std::pair<double, int>> tot;
  for (int k = 0; k < nb; ++k) {
    const unsigned long long* r = &t[kTickSlots * static_cast<size_t>(k)];
    const int mode = static_cast<int>(r[6] & 3);
    double ph[4] = {double(r[1] - r[0]), double(r[2] - r[1]), double(r[3] - r[2]),
                    double(r[4] - r[3])};
    for (int q = 0; q < 4; ++q) sum[mode][q] += ph[q];
    sum[mode][4] = std::max(sum[mode][4], double(r[4] - r[0]));
    ++cnt[mode];
    t_first = std::min(t_first, r[0]);
    t_last = std::max(t_last, r[4]);
    tot.emplace_back(double(r[4] - r[0]), k);
  }
  std::sort(tot.begin(), tot.end(), [](auto& a, auto& b) { return a.first > b.first; });
  std::fprintf(stderr, "[blocks from %d] %d blocks, span %llu ticks\n", first, nb,
               t_last - t_first);
  for (int m = 0; m < 3; ++m)
    if (cnt[m])
      std::fprintf(stderr, "   mode %d: %d blocks; sum assemble %.3g factor %.3g normalise %.3g "
                   "substitute %.3g; slowest %.3g\n", m, cnt[m], sum[m][0], sum[m][1], sum[m][2],
                   sum[m][3], sum[m][4]);
  for (int q = 0; q < std::min(nb, 6); ++q) {
    const unsigned long long* r = &t[kTickSlots * static_cast<size_t>(tot[q].second)];
    std::fprintf(stderr, "   n %llu b %llu nck %llu mode %llu : assemble %llu factor %llu normalise %llu substitute %llu\n",
                 r[5] >> 32, r[5] & 0xffffffffull, r[6] >> 32, r[6] & 0xffffffffull, r[1] - r[0],
                 r[2] - r[1], r[3] - r[2], r[4] - r[3]);
    if (r[8] | r[9] | r[10] | r[11] | r[12])
      std::fprintf(stderr, "      blocked factor: ring load %llu panel %llu D/L %llu trailing %llu ring store %llu\n",
                   r[8], r[9], r[10], r[11], r[12]);
  }
}

namespace {

// ---- MSFV / MSMIX restriction (Sec. 3, 3.2) --------------------------------
__global__ void k_block_count(int n, int nc, const int* primal, int* cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&cnt[primal[i]], 1);
}

__global__ void k_iota_r(int n, int* v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = i;
}

// row i takes the primal block's cells (MSFV) or keeps its row of P^T
__device__ __forceinline__ bool fv_row(int i, int restriction, int nm, const int* vertex) {
  return restriction == FAMS_RESTRICT_FV || vertex[i] >= nm;
}

__global__ void k_r_counts(int nc, int restriction, int nm, const int* vertex, const int* bptr,
                           const int* r_rp, int* cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nc)
    cnt[i] = fv_row(i, restriction, nm, vertex) ? bptr[i + 1] - bptr[i] : r_rp[i + 1] - r_rp[i];
  if (i == nc) cnt[nc] = 0;
}

__global__ void k_r_rows(int nc, int restriction, int nm, const int* vertex, const int* bptr,
                         const int* cells, const int* r_rp, const int* r_ci, const double* r_val,
                         const int* nrp, int* nci, double* nval) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  int o = nrp[i];
  if (fv_row(i, restriction, nm, vertex)) {
    for (int t = bptr[i]; t < bptr[i + 1]; ++t, ++o) {
      nci[o] = cells[t];
      nval[o] = 1.0;
    }
  } else {
    for (int p = r_rp[i]; p < r_rp[i + 1]; ++p, ++o) {
      nci[o] = r_ci[p];
      nval[o] = r_val[p];
    }
  }
}

}  // namespace

// R^FV: row i has a 1 on every cell of primal block i (the cells in
// ascending order, from a stable sort by block); MSMIX takes these rows for
// the coarse nodes whose vertex is a fracture cell and keeps the rows of
// P^T for the matrix ones.  Replaces R (and its FP32 copy).
void build_restriction(Handle* h) {
  const int n = h->n, nc = h->nc;
  Allocator* A = &h->alloc;
  DBuf<int> cnt(A, nc + 1), bptr(A, nc + 1), keys(A, n), iota(A, n), cells(A, n);
  HIPX(hipMemsetAsync(cnt, 0, (nc + 1) * sizeof(int), h->stream));
  LAUNCH(h, "r_blocks", k_block_count, blocks_for(n, kThreads), kThreads, 0, n, nc,
         h->primal.get(), cnt.get());
  exclusive_scan_i32(h, cnt, bptr, nc + 1);
  LAUNCH(h, "r_blocks", k_iota_r, blocks_for(n, kThreads), kThreads, 0, n, iota.get());
  sort_pairs_i32(h, h->primal, keys, iota, cells, n, bits_for(nc));
  LAUNCH(h, "r_rows", k_r_counts, blocks_for(nc + 1, kThreads), kThreads, 0, nc, h->restriction,
         h->nm, h->vertex.get(), bptr.get(), h->r_rp.get(), cnt.get());
  DBuf<int> nrp(A, nc + 1);
  exclusive_scan_i32(h, cnt, nrp, nc + 1);
  int nnz = 0;
  HIPX(hipMemcpyAsync(&nnz, nrp.get() + nc, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  DBuf<int> nci(A, std::max(nnz, 1));
  DBuf<double> nval(A, std::max(nnz, 1));
  LAUNCH(h, "r_rows", k_r_rows, blocks_for(nc, kThreads), kThreads, 0, nc, h->restriction, h->nm,
         h->vertex.get(), bptr.get(), cells.get(), h->r_rp.get(), h->r_ci.get(),
         h->r_val.get(), nrp.get(), nci.get(), nval.get());
  HIPX(hipStreamSynchronize(h->stream));
  h->r_rp = std::move(nrp);
  h->r_ci = std::move(nci);
  h->r_val = std::move(nval);
  if (h->precision == FAMS_PREC_MIXED) {
    h->r_val32.reset(A, std::max(nnz, 1));
    LAUNCH(h, "d2f", k_d2f, blocks_for(nnz, kThreads), kThreads, 0, static_cast<int64_t>(nnz),
           h->r_val.get(), h->r_val32.get());
  }
  HIPX(hipStreamSynchronize(h->stream));
}

void build_prolongation(Handle* h, const int8_t* wb) {
  const int n = h->n, nm = h->nm, nc = h->nc, nwb = h->n - h->nw;
  unsigned g = blocks_for(n, kThreads);
  Allocator* A = &h->alloc;
  PhaseTimer pt(h->stream);
  h->info.local_flops = 0;  // counted afresh for every basis
  h->info.local_subst_flops = 0;

  DBuf<int> coarse_of(A, n), err(A, 1);
  DBuf<int8_t> rho(A, n), ecls(A, h->nnz);
  HIPX(hipMemsetAsync(coarse_of, 0xff, n * sizeof(int), h->stream));
  HIPX(hipMemsetAsync(err, 0, sizeof(int), h->stream));
  // the validate kernel reads vertex as int64 from the handle's int copy
  DBuf<int64_t> vtx64(A, nc);
  {
    std::vector<int> hv(nc);
    HIPX(hipMemcpyAsync(hv.data(), h->vertex.get(), nc * sizeof(int), hipMemcpyDeviceToHost,
                        h->stream));
    HIPX(hipStreamSynchronize(h->stream));
    std::vector<int64_t> hv64(hv.begin(), hv.end());
    HIPX(hipMemcpyAsync(vtx64, hv64.data(), nc * sizeof(int64_t), hipMemcpyHostToDevice,
                        h->stream));
  }
  LAUNCH(h, "validate", k_validate, blocks_for(std::max(n, nc), kThreads), kThreads, 0, n, nm,
         nwb, nc, wb, h->primal.get(), vtx64.get(), coarse_of.get(), rho.get(), h->variant,
         err.get());
  LAUNCH(h, "check_vertices", k_check_vertices, g, kThreads, 0, n, wb, coarse_of.get(), err.get());
  int e = static_cast<int>(read1(h, err.get()));
  FAMS_REQUIRE(e == 0, FAMS_ERR_BAD_GRID, grid_error_text(e));

  // entry classes and local blocks
  DBuf<int> label(A, n);
  if (h->variant == FAMS_COUPLED) {
    LAUNCH(h, "classify", k_classify, g, kThreads, 0, n, nm, nwb, h->rp.get(), h->ci.get(), wb,
           rho.get(), static_cast<int>(FAMS_DECOUPLED), static_cast<const int*>(nullptr),
           ecls.get());
    DBuf<int> base(A, n);
    components(h, wb, ecls, base);
    coupled_groups(h, wb, base, label);
    LAUNCH(h, "classify", k_classify, g, kThreads, 0, n, nm, nwb, h->rp.get(), h->ci.get(), wb,
           rho.get(), static_cast<int>(FAMS_COUPLED), static_cast<const int*>(label.get()),
           ecls.get());
  } else {
    LAUNCH(h, "classify", k_classify, g, kThreads, 0, n, nm, nwb, h->rp.get(), h->ci.get(), wb,
           rho.get(), h->variant, static_cast<const int*>(nullptr), ecls.get());
    components(h, wb, ecls, label);
  }

  // blocks in level order (rank descending, then ascending root cell)
  DBuf<int> flag(A, n), pos(A, n);
  LAUNCH(h, "root_flags", k_root_flags, g, kThreads, 0, n, label.get(), flag.get());
  exclusive_scan_i32(h, flag, pos, n);
  const int ncomp = static_cast<int>(read1(h, pos.get() + n - 1) + read1(h, flag.get() + n - 1));
  FAMS_REQUIRE(ncomp > 0 || n == nc, FAMS_ERR_BAD_GRID, "no non-vertex cells");
  DBuf<int> ck(A, std::max(ncomp, 1)), cv(A, std::max(ncomp, 1)), cks(A, std::max(ncomp, 1)),
      cvs(A, std::max(ncomp, 1)), croot(A, n);
  LAUNCH(h, "root_keys", k_root_keys, g, kThreads, 0, n, label.get(), rho.get(), pos.get(),
         ck.get(), cv.get());
  sort_pairs_i32(h, ck, cks, cv, cvs, ncomp, 3);
  LAUNCH(h, "comp_index", k_comp_index, blocks_for(ncomp, kThreads), kThreads, 0, ncomp, cvs.get(),
         croot.get());
  DBuf<int> comp_of(A, n);
  LAUNCH(h, "comp_of", k_comp_of, g, kThreads, 0, n, label.get(), croot.get(), comp_of.get(),
         flag.get());
  exclusive_scan_i32(h, flag, pos, n);
  const int m = n - nc;  // non-vertex cells
  DBuf<int> kk(A, std::max(m, 1)), kv(A, std::max(m, 1)), kks(A, std::max(m, 1)),
      cells(A, std::max(m, 1));
  LAUNCH(h, "cell_keys", k_cell_keys, g, kThreads, 0, n, comp_of.get(), pos.get(), kk.get(),
         kv.get());
  sort_pairs_i32(h, kk, kks, kv, cells, m, bits_for(ncomp));
  DBuf<int> comp_ptr(A, ncomp + 1), local_idx(A, n);
  if (m) {
    LAUNCH(h, "comp_ptr", k_comp_ptr, blocks_for(m, kThreads), kThreads, 0, m, ncomp, kks.get(),
           cells.get(), comp_ptr.get(), local_idx.get());
    LAUNCH(h, "local_idx", k_local_idx, blocks_for(m, kThreads), kThreads, 0, m, kks.get(),
           cells.get(), comp_ptr.get(), local_idx.get());
  }
  if (ncomp) {
    const int cap = order_adj_cap(lds_hw_budget(h));
    allow_lds(reinterpret_cast<const void*>(&k_local_order<KeptEdge>),
              cap * sizeof(unsigned short));
    LAUNCH(h, "local_order", k_local_order<KeptEdge>, ncomp, kOrderThreads,
           cap * sizeof(unsigned short), comp_ptr.get(), cells.get(), h->rp.get(), h->ci.get(),
           KeptEdge{ecls.get()}, local_idx.get(), cap);
  }
  std::vector<int> h_cks(ncomp), h_comp_ptr(ncomp + 1, 0);
  if (ncomp) {
    HIPX(hipMemcpyAsync(h_cks.data(), cks.get(), ncomp * sizeof(int), hipMemcpyDeviceToHost,
                        h->stream));
    HIPX(hipMemcpyAsync(h_comp_ptr.data(), comp_ptr.get(), (ncomp + 1) * sizeof(int),
                        hipMemcpyDeviceToHost, h->stream));
  }
  HIPX(hipStreamSynchronize(h->stream));
  {  // blocks too large for the LDS ordering (kOrderMax < n <= 32768)
    int big = 0;
    for (int K = 0; K < ncomp; ++K) {
      const int nk = h_comp_ptr[K + 1] - h_comp_ptr[K];
      if (nk > kOrderMax && nk <= 32768) big = std::max(big, nk);
    }
    if (big) {
      DBuf<int> lvl(A, big), keys(A, big), vals(A, big), keys_s(A, big), vals_s(A, big),
          info(A, 1);
      for (int K = 0; K < ncomp; ++K) {
        const int nk = h_comp_ptr[K + 1] - h_comp_ptr[K];
        if (nk <= kOrderMax || nk > 32768) continue;
        LAUNCH(h, "local_order", k_bfs_levels<KeptEdge>, 1, kThreads, 0, K, h_comp_ptr[K], nk,
               cells.get(), h->rp.get(), h->ci.get(), KeptEdge{ecls.get()}, local_idx.get(),
               lvl.get(), keys.get(), vals.get(), info.get());
        sort_pairs_i32(h, keys, keys_s, vals, vals_s, nk, 31);
        LAUNCH(h, "local_order", k_apply_order<KeptEdge>, 1, kThreads, 0, K, h_comp_ptr[K], nk,
               cells.get(), h->rp.get(), h->ci.get(), KeptEdge{ecls.get()}, local_idx.get(),
               keys_s.get(), vals_s.get(), lvl.get(), info.get());
      }
      HIPX(hipStreamSynchronize(h->stream));
    }
  }
  // level ranges (key = 7 - rank)
  std::vector<std::pair<int, int>> levels;
  for (int k = 0; k < ncomp;) {
    int e2 = k;
    while (e2 < ncomp && h_cks[e2] == h_cks[k]) ++e2;
    levels.emplace_back(k, e2);
    k = e2;
  }
  int max_block = 0;
  for (int k = 0; k < ncomp; ++k) max_block = std::max(max_block, h_comp_ptr[k + 1] - h_comp_ptr[k]);
  h->info.n_blocks = ncomp;
  h->info.max_block = max_block;

  // symbolic: coarse columns per block, level by level
  DBuf<int> ncols(A, std::max(ncomp, 1)), band(A, std::max(ncomp, 1));
  DBuf<int64_t> col_ptr(A, ncomp + 1);
  std::vector<int64_t> h_col_ptr(ncomp + 1, 0);
  std::vector<int> h_ncols(ncomp, 0), h_band(ncomp, 0);
  DBuf<int> cols(A, 1);
  int64_t cols_size = 0;
  HIPX(hipMemsetAsync(col_ptr, 0, (ncomp + 1) * sizeof(int64_t), h->stream));
  DBuf<int> diag(A, 4);
  HIPX(hipMemsetAsync(diag, 0xff, 4 * sizeof(int), h->stream));
  for (auto [c0, c1] : levels) {
    int nl = c1 - c0;
    DBuf<int> tmp(A, static_cast<size_t>(nl) * kMaxCols);
    LAUNCH(h, "colset", k_colset, nl, kThreads, 0, c0, comp_ptr.get(), cells.get(), h->rp.get(),
           h->ci.get(), ecls.get(), wb, coarse_of.get(), comp_of.get(), local_idx.get(),
           col_ptr.get(), cols.get(), tmp.get(), ncols.get(), band.get(), err.get(), diag.get());
    HIPX(hipMemcpyAsync(h_ncols.data() + c0, ncols.get() + c0, nl * sizeof(int),
                        hipMemcpyDeviceToHost, h->stream));
    HIPX(hipMemcpyAsync(h_band.data() + c0, band.get() + c0, nl * sizeof(int),
                        hipMemcpyDeviceToHost, h->stream));
    int ev = static_cast<int>(read1(h, err.get()));
    FAMS_REQUIRE(!(ev & E_NO_HIGHER), FAMS_ERR_SINGULAR_LOCAL,
                 "a local block has no higher-rank neighbour");
    if (ev & (E_SOURCES | E_COLS)) {
      int hd[4];
      HIPX(hipMemcpyAsync(hd, diag.get(), sizeof(hd), hipMemcpyDeviceToHost, h->stream));
      HIPX(hipStreamSynchronize(h->stream));
      throw Error(FAMS_ERR_CAPACITY,
                  "local block " + std::to_string(hd[0]) + " (" + std::to_string(hd[2]) +
                      " cells, " + std::to_string(hd[1]) + " higher-rank couplings/sources, " +
                      std::to_string(hd[3]) + " columns) exceeds a per-block limit (flags " +
                      std::to_string(ev) + ")");
    }
    for (int K = c0; K < c1; ++K) h_col_ptr[K + 1] = h_col_ptr[K] + h_ncols[K];
    int64_t new_size = h_col_ptr[c1];
    DBuf<int> grown(A, std::max<int64_t>(new_size, 1));
    if (cols_size)
      HIPX(hipMemcpyAsync(grown, cols.get(), cols_size * sizeof(int), hipMemcpyDeviceToDevice,
                          h->stream));
    HIPX(hipMemcpyAsync(col_ptr.get() + c0 + 1, h_col_ptr.data() + c0 + 1, nl * sizeof(int64_t),
                        hipMemcpyHostToDevice, h->stream));
    LAUNCH(h, "colcopy", k_colcopy, nl, kThreads, 0, c0, nl, tmp.get(), col_ptr.get(),
           grown.get());
    HIPX(hipStreamSynchronize(h->stream));
    cols = std::move(grown);
    cols_size = new_size;
  }

  pt.mark("blocks + column sets");
  // numeric: solve the blocks level by level
  std::vector<int64_t> h_pval_off(ncomp + 1, 0);
  for (int K = 0; K < ncomp; ++K)
    h_pval_off[K + 1] =
        h_pval_off[K] + static_cast<int64_t>(h_comp_ptr[K + 1] - h_comp_ptr[K]) * h_ncols[K];
  DBuf<int64_t> pval_off(A, ncomp + 1);
  HIPX(hipMemcpyAsync(pval_off, h_pval_off.data(), (ncomp + 1) * sizeof(int64_t),
                      hipMemcpyHostToDevice, h->stream));
  const bool mixed = h->precision == FAMS_PREC_MIXED;
  DBuf<double> pv64;
  DBuf<float> pv32;
  DBuf<int> bad_block;
  if (mixed) {
    pv32.reset(A, std::max<int64_t>(h_pval_off[ncomp], 1));
    bad_block.reset(A, std::max(ncomp, 1));
    HIPX(hipMemsetAsync(bad_block, 0, std::max(ncomp, 1) * sizeof(int), h->stream));
  } else {
    pv64.reset(A, std::max<int64_t>(h_pval_off[ncomp], 1));
  }
  int64_t fallbacks = 0;
  // FAMS_FORCE_FP64_BLOCKS=k (tests): in the precision form, blocks whose id
  // is a multiple of k also take the FP64 re-solve, as if their FP32
  // factorisation had met a non-positive pivot
  int force_k = 0;
  if (const char* e = std::getenv("FAMS_FORCE_FP64_BLOCKS")) force_k = std::max(0, std::atoi(e));
  for (auto [c0, c1] : levels) {
    HIPX(hipMemsetAsync(err, 0, sizeof(int), h->stream));
    std::vector<int> blocks(c1 - c0);
    std::iota(blocks.begin(), blocks.end(), c0);
    if (mixed) {
      local_solves<float, float>(h, blocks, false, comp_ptr, cells, ecls, wb, coarse_of, comp_of,
                                 local_idx, col_ptr, cols, ncols, band, pval_off, pv32.get(),
                                 h_comp_ptr, h_band, h_ncols, err, bad_block);
    } else {
      local_solves<double, double>(h, blocks, false, comp_ptr, cells, ecls, wb, coarse_of,
                                   comp_of, local_idx, col_ptr, cols, ncols, band, pval_off,
                                   pv64.get(), h_comp_ptr, h_band, h_ncols, err, nullptr);
    }
    int ev = static_cast<int>(read1(h, err.get()));
    if (mixed && ((ev & E_PIVOT) || force_k > 0)) {
      // FP32 breakdown: re-solve the affected blocks of this level in FP64
      std::vector<int> hb(c1 - c0);
      HIPX(hipMemcpyAsync(hb.data(), bad_block.get() + c0, (c1 - c0) * sizeof(int),
                          hipMemcpyDeviceToHost, h->stream));
      HIPX(hipStreamSynchronize(h->stream));
      std::vector<int> redo;
      for (int k = 0; k < c1 - c0; ++k)
        if (hb[k] || (force_k > 0 && (c0 + k) % force_k == 0)) redo.push_back(c0 + k);
      fallbacks += static_cast<int64_t>(redo.size());
      if (!redo.empty()) {
        HIPX(hipMemsetAsync(err, 0, sizeof(int), h->stream));
        local_solves<float, double>(h, redo, true, comp_ptr, cells, ecls, wb, coarse_of, comp_of,
                                    local_idx, col_ptr, cols, ncols, band, pval_off, pv32.get(),
                                    h_comp_ptr, h_band, h_ncols, err, nullptr);
        ev = static_cast<int>(read1(h, err.get()));
      }
    }
    FAMS_REQUIRE(!(ev & E_PIVOT), FAMS_ERR_SINGULAR_LOCAL, "non-positive pivot in a local block");
    pt.mark("local solves (level)");
  }
  h->info.fp32_fallback_blocks = fallbacks;

  // P as CSR (truncated), then R = P^T by a stable sort on the column
  h->pell.clear();  // the lock-step products' fixed-width copy follows P
  DBuf<int> cnt(A, n);
  h->p_rp.reset(A, n + 1);
  if (mixed)
    LAUNCH(h, "p_count", k_p_count<float>, g, kThreads, 0, n, wb, comp_of.get(), local_idx.get(),
           ncols.get(), pval_off.get(), static_cast<const float*>(pv32.get()), h->alpha,
           cnt.get());
  else
    LAUNCH(h, "p_count", k_p_count<double>, g, kThreads, 0, n, wb, comp_of.get(), local_idx.get(),
           ncols.get(), pval_off.get(), static_cast<const double*>(pv64.get()), h->alpha,
           cnt.get());
  exclusive_scan_i32(h, cnt, h->p_rp, n);
  int64_t pnnz = read1(h, h->p_rp.get() + n - 1) + read1(h, cnt.get() + n - 1);
  FAMS_REQUIRE(pnnz < (int64_t(1) << 31), FAMS_ERR_CAPACITY, "nnz(P) >= 2^31");
  {
    int v = static_cast<int>(pnnz);
    HIPX(hipMemcpyAsync(h->p_rp.get() + n, &v, sizeof(int), hipMemcpyHostToDevice, h->stream));
    HIPX(hipStreamSynchronize(h->stream));
  }
  h->p_nnz = pnnz;
  h->p_ci.reset(A, pnnz);
  h->p_val.reset(A, pnnz);
  if (mixed)
    LAUNCH(h, "p_fill", k_p_fill<float>, g, kThreads, 0, n, wb, coarse_of.get(), comp_of.get(),
           local_idx.get(), ncols.get(), col_ptr.get(), cols.get(), pval_off.get(),
           static_cast<const float*>(pv32.get()), h->alpha, h->p_rp.get(), h->p_ci.get(),
           h->p_val.get());
  else
    LAUNCH(h, "p_fill", k_p_fill<double>, g, kThreads, 0, n, wb, coarse_of.get(), comp_of.get(),
           local_idx.get(), ncols.get(), col_ptr.get(), cols.get(), pval_off.get(),
           static_cast<const double*>(pv64.get()), h->alpha, h->p_rp.get(), h->p_ci.get(),
           h->p_val.get());
  h->info.nnz_P = pnnz;

  DBuf<int> erow(A, pnnz), iota(A, pnnz), keys(A, pnnz), perm(A, pnnz);
  LAUNCH(h, "entry_rows", k_entry_rows, g, kThreads, 0, n, h->p_rp.get(), erow.get(), iota.get());
  sort_pairs_i32(h, h->p_ci, keys, iota, perm, pnnz, bits_for(nc));
  h->r_rp.reset(A, nc + 1);
  h->r_ci.reset(A, pnnz);
  h->r_val.reset(A, pnnz);
  LAUNCH(h, "r_fill", k_r_fill, blocks_for(pnnz, kThreads), kThreads, 0, pnnz, nc, keys.get(),
         perm.get(), erow.get(), h->p_val.get(), h->r_rp.get(), h->r_ci.get(), h->r_val.get());
  if (mixed) {
    h->p_val32.reset(A, pnnz);
    h->r_val32.reset(A, pnnz);
    LAUNCH(h, "d2f", k_d2f, blocks_for(pnnz, kThreads), kThreads, 0, pnnz, h->p_val.get(),
           h->p_val32.get());
    LAUNCH(h, "d2f", k_d2f, blocks_for(pnnz, kThreads), kThreads, 0, pnnz, h->r_val.get(),
           h->r_val32.get());
  }
  HIPX(hipStreamSynchronize(h->stream));
  pt.mark("P and R");
}

}  // namespace fams
