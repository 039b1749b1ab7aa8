// Block-local helpers shared by the basis blocks and the primal blocks of the
// flux reconstruction: a workgroup-wide bitonic sort and the breadth-first
// local ordering that narrows the band of irregular blocks.
#pragma once

#include <hip/hip_runtime.h>

namespace fams {
namespace {

__device__ inline void block_bitonic_sort(int* a, int cnt) {
  int m = 1;
  while (m < cnt) m <<= 1;
  for (int t = cnt + threadIdx.x; t < m; t += blockDim.x) a[t] = INT_MAX;
  __syncthreads();
  for (int k = 2; k <= m; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < m; t += blockDim.x) {
        int u = t ^ j;
        if (u > t) {
          bool up = (t & k) == 0;
          int x = a[t], y = a[u];
          if ((x > y) == up) {
            a[t] = y;
            a[u] = x;
          }
        }
      }
      __syncthreads();
    }
  }
}

// exclusive prefix sum of a[0, cnt) in place (LDS); a[cnt] receives the
// total.  s_part holds blockDim.x + 1 ints; every thread of the block calls it.
__device__ inline void block_exclusive_scan(int* a, int cnt, int* s_part) {
  const int T = blockDim.x, tid = threadIdx.x;
  const int per = (cnt + T - 1) / T, b = min(cnt, tid * per), e = min(cnt, b + per);
  int sum = 0;
  for (int l = b; l < e; ++l) sum += a[l];
  s_part[tid] = sum;
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int t = 0; t < T; ++t) {
      const int v = s_part[t];
      s_part[t] = run;
      run += v;
    }
    s_part[T] = run;
  }
  __syncthreads();
  int run = s_part[tid];
  for (int l = b; l < e; ++l) {
    const int v = a[l];
    a[l] = run;
    run += v;
  }
  if (tid == 0) a[cnt] = s_part[T];
  __syncthreads();
}

// Local order of a block: breadth-first levels from a pseudo-peripheral cell,
// cells of one level by ascending natural position.  Irregular blocks (fracture
// regions, merged Coupled-AMS blocks) get a bandwidth tens of times smaller
// than in ascending-index order; structured dual blocks keep their natural
// order, which is narrower for them.  The order used is the narrower one.
// `edge(p, i, K)` tells whether CSR entry p of row i couples two cells of
// block K (the block's own couplings).  The block's couplings are first
// staged in LDS as a local adjacency (16-bit local indices, at most adj_cap
// of them, in the dynamic LDS), so the breadth-first levels and both
// bandwidth measurements read LDS only; a block with more couplings reads
// them from the CSR each time.
constexpr int kOrderMax = 6144;
constexpr int kOrderThreads = 256;
constexpr int kOrderStaticBytes = (kOrderMax + 8192 + kOrderMax + 1 + kOrderThreads + 1 + 4) * 4;
constexpr int kOrderAdjMax = 40960;

// couplings a block can stage, given the LDS of one workgroup (bytes)
inline int order_adj_cap(int64_t lds_bytes) {
  const int64_t room = (lds_bytes - kOrderStaticBytes - 256) / 2;
  return static_cast<int>(room < 0 ? 0 : (room > kOrderAdjMax ? kOrderAdjMax : room));
}

template <class Edge>
__global__ void __launch_bounds__(kOrderThreads)
k_local_order(const int* comp_ptr, int* cells, const int* rp, const int* ci, Edge edge,
              int* local_idx, int adj_cap) {
  __shared__ int lvl[kOrderMax];
  __shared__ int key[8192];
  __shared__ int s_off[kOrderMax + 1];
  __shared__ int s_part[kOrderThreads + 1];
  __shared__ int s_changed, s_bnat, s_bbfs, s_start;
  extern __shared__ unsigned short s_adj[];
  int K = blockIdx.x;
  int beg = comp_ptr[K], n = comp_ptr[K + 1] - beg;
  if (n <= 2 || n > kOrderMax) return;
  if (threadIdx.x == 0) {
    s_bnat = 0;
    s_bbfs = 0;
  }
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    const int i = cells[beg + l];
    int cnt = 0;
    for (int p = rp[i]; p < rp[i + 1]; ++p)
      if (edge(p, i, K)) ++cnt;
    s_off[l] = cnt;
  }
  __syncthreads();
  block_exclusive_scan(s_off, n, s_part);
  const bool staged = s_off[n] <= adj_cap;
  if (staged) {
    for (int l = threadIdx.x; l < n; l += blockDim.x) {
      const int i = cells[beg + l];
      int o = s_off[l];
      for (int p = rp[i]; p < rp[i + 1]; ++p)
        if (edge(p, i, K)) s_adj[o++] = static_cast<unsigned short>(local_idx[ci[p]]);
    }
    __syncthreads();
  }
  // f(local index) for every coupling of local cell l
  auto for_nbrs = [&](int l, auto f) {
    if (staged) {
      for (int o = s_off[l]; o < s_off[l + 1]; ++o) f(static_cast<int>(s_adj[o]));
    } else {
      const int i = cells[beg + l];
      for (int p = rp[i]; p < rp[i + 1]; ++p)
        if (edge(p, i, K)) f(local_idx[ci[p]]);
    }
  };
  int bnat = 0;
  for (int l = threadIdx.x; l < n; l += blockDim.x)
    for_nbrs(l, [&](int lj) { bnat = max(bnat, abs(lj - l)); });
  atomicMax(&s_bnat, bnat);
  // Two breadth-first passes: the second starts from the lowest cell of the
  // first pass's last level (a pseudo-peripheral cell), which narrows the
  // levels of elongated blocks.
  int start = 0;
  for (int pass = 0; pass < 2; ++pass) {
    for (int l = threadIdx.x; l < n; l += blockDim.x) lvl[l] = l == start ? 0 : -1;
    __syncthreads();
    int last = 0;
    for (int d = 0; d < n; ++d) {
      if (threadIdx.x == 0) s_changed = 0;
      __syncthreads();
      for (int l = threadIdx.x; l < n; l += blockDim.x) {
        if (lvl[l] != d) continue;
        for_nbrs(l, [&](int lj) {
          if (lvl[lj] < 0) {
            lvl[lj] = d + 1;
            s_changed = 1;
          }
        });
      }
      __syncthreads();
      const int changed = s_changed;
      __syncthreads();  // every thread has read the flag before it is reset
      if (!changed) {
        last = d;
        break;
      }
    }
    if (pass == 0) {
      if (threadIdx.x == 0) s_start = n;
      __syncthreads();
      for (int l = threadIdx.x; l < n; l += blockDim.x)
        if (lvl[l] == last) atomicMin(&s_start, l);
      __syncthreads();
      start = s_start;
      __syncthreads();
    }
  }
  for (int l = threadIdx.x; l < n; l += blockDim.x) key[l] = (lvl[l] << 13) | l;
  __syncthreads();
  block_bitonic_sort(key, n);
  for (int t = threadIdx.x; t < n; t += blockDim.x) lvl[key[t] & 8191] = t;  // lvl := position
  __syncthreads();
  int bb = 0;
  for (int l = threadIdx.x; l < n; l += blockDim.x)
    for_nbrs(l, [&](int lj) { bb = max(bb, abs(lvl[lj] - lvl[l])); });
  atomicMax(&s_bbfs, bb);
  __syncthreads();
  if (s_bbfs >= s_bnat) return;
  for (int l = threadIdx.x; l < n; l += blockDim.x) key[l] = cells[beg + l];
  __syncthreads();
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    cells[beg + lvl[l]] = key[l];
    local_idx[key[l]] = lvl[l];
  }
}
template <class Edge>
__global__ void __launch_bounds__(256)
k_bfs_levels(int K, int beg, int n, const int* cells, const int* rp, const int* ci, Edge edge,
             const int* local_idx, int* lvl, int* keys, int* vals, int* info) {
  __shared__ int s_changed, s_start, s_bnat;
  if (threadIdx.x == 0) s_bnat = 0;
  __syncthreads();
  int bnat = 0;
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    const int i = cells[beg + l];
    for (int p = rp[i]; p < rp[i + 1]; ++p)
      if (edge(p, i, K)) bnat = max(bnat, abs(local_idx[ci[p]] - l));
  }
  atomicMax(&s_bnat, bnat);
  int start = 0;
  for (int pass = 0; pass < 2; ++pass) {
    for (int l = threadIdx.x; l < n; l += blockDim.x) lvl[l] = l == start ? 0 : -1;
    __syncthreads();
    int last = 0;
    for (int d = 0; d < n; ++d) {
      if (threadIdx.x == 0) s_changed = 0;
      __syncthreads();
      for (int l = threadIdx.x; l < n; l += blockDim.x) {
        if (lvl[l] != d) continue;
        const int i = cells[beg + l];
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
          if (!edge(p, i, K)) continue;
          const int lj = local_idx[ci[p]];
          if (lvl[lj] < 0) {
            lvl[lj] = d + 1;
            s_changed = 1;
          }
        }
      }
      __syncthreads();
      const int changed = s_changed;
      __syncthreads();
      if (!changed) {
        last = d;
        break;
      }
    }
    if (pass == 0) {
      if (threadIdx.x == 0) s_start = n;
      __syncthreads();
      for (int l = threadIdx.x; l < n; l += blockDim.x)
        if (lvl[l] == last) atomicMin(&s_start, l);
      __syncthreads();
      start = s_start;
      __syncthreads();
    }
  }
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    keys[l] = (max(lvl[l], 0) << 16) | l;   // unreached cells (none in a component) first
    vals[l] = cells[beg + l];
  }
  if (threadIdx.x == 0) info[0] = s_bnat;
}

// apply the sorted order if it is narrower than the natural one
template <class Edge>
__global__ void __launch_bounds__(256)
k_apply_order(int K, int beg, int n, int* cells, const int* rp, const int* ci, Edge edge,
              int* local_idx, const int* keys_s, const int* vals_s, int* pos, const int* info) {
  __shared__ int s_bb;
  if (threadIdx.x == 0) s_bb = 0;
  for (int t = threadIdx.x; t < n; t += blockDim.x) pos[keys_s[t] & 0xFFFF] = t;
  __syncthreads();
  int bb = 0;
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    const int i = cells[beg + l];
    for (int p = rp[i]; p < rp[i + 1]; ++p)
      if (edge(p, i, K)) bb = max(bb, abs(pos[local_idx[ci[p]]] - pos[l]));
  }
  atomicMax(&s_bb, bb);
  __syncthreads();
  if (s_bb >= info[0]) return;
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    cells[beg + t] = vals_s[t];
    local_idx[vals_s[t]] = t;
  }
}

}  // namespace
}  // namespace fams
