// ILU(0) smoother of Table 1 step 7 (Sec. 3.2): incomplete LU of A on A's own
// sparsity pattern, rows in their given (natural) order, and its application
// x = U^{-1} L^{-1} b by level-scheduled triangular sweeps.
//
// Level of row i in the lower sweep = 1 + max level of the rows j < i it
// depends on (0 if none); the upper sweep uses j > i.  The factorisation runs
// one launch per level (a thread per row).  Each sweep of the iteration is a
// single launch that walks the rows in level order and lets every row wait
// only for its own dependencies (see k_sweep_lower).  The natural ordering --
// and hence the smoother itself -- is unchanged.
#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <type_traits>
#include <vector>

#include "band.hpp"
#include "internal.hpp"

namespace fams {
namespace {

constexpr int kT = 256;
constexpr int kSweepGroups = 256;  // workgroups of a one-launch sweep

__global__ void k_diag_pos(int n, const int* rp, const int* ci, int* diag, int* err) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int d = -1;
  for (int p = rp[i]; p < rp[i + 1]; ++p)
    if (ci[p] == i) d = p;
  diag[i] = d;
  if (d < 0) atomicOr(err, 1);
}

__global__ void k_iota(int n, int* v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = i;
}

__global__ void k_level_ptr(int n, const int* key_sorted, int* ptr) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  int k = key_sorted[t];
  if (t == 0 || key_sorted[t - 1] != k) ptr[k] = t;
  if (t == n - 1) ptr[k + 1] = n;
}

// ---- dataflow over natural-order chunks ----------------------------------------
// Dependency levels in one launch per triangle: a workgroup takes the next
// chunk of 256 consecutive rows (ascending for the lower triangle, descending
// for the upper one) from a ticket; every dependency of a row lies in the same
// or an earlier chunk.  A lane never spins on its own: each pass of the loop
// either finishes its row (all dependencies published) or leaves it for the
// next pass, so a row that depends on a row of the same wavefront is finished
// one pass after it.  The loop is bounded by the wall-clock limit and the
// shared error flag, like the sweeps.
constexpr int kLevDeps = 8;

template <bool kUpper>
__global__ void __launch_bounds__(256)
k_levels_df(int n, const int* rp, const int* ci, const int* diag, int* lev, int* ticket,
            int* err, unsigned long long limit) {
  __shared__ int s_c;
  const int nchunks = (n + 255) / 256;
  while (true) {
    if (threadIdx.x == 0) s_c = atomicAdd(ticket, 1);
    __syncthreads();
    const int c = s_c;
    __syncthreads();
    if (c >= nchunks) break;
    const int i = kUpper ? n - 1 - (c * 256 + static_cast<int>(threadIdx.x))
                         : c * 256 + static_cast<int>(threadIdx.x);
    bool done = i < 0 || i >= n;
    const int p0 = done ? 0 : (kUpper ? diag[i] + 1 : rp[i]);
    const int p1 = done ? 0 : (kUpper ? rp[i + 1] : diag[i]);
    const unsigned long long t0 = wall_clock64();
    // a row of at most kLevDeps dependencies keeps their columns in registers
    // and, pass by pass, reloads only the levels it has not seen yet
    const bool few = p1 - p0 <= kLevDeps;
    int dep[kLevDeps];
    unsigned pending = 0;
#pragma unroll
    for (int k = 0; k < kLevDeps; ++k)
      if (few && p0 + k < p1) {
        dep[k] = ci[p0 + k];
        pending |= 1u << k;
      }
    int Lk = 0;  // level bound from the dependencies seen so far (few)
    // the exit test is a wavefront vote, so a lane that finishes publishes in
    // the pass where it finishes (no lane leaves the loop on its own, which
    // would let the compiler move the store past the loop)
    while (__any(!done)) {
      if (!done) {
        int L = 0;
        bool ready = true;
        if (few) {
          int v[kLevDeps];
#pragma unroll
          for (int k = 0; k < kLevDeps; ++k)
            if (pending >> k & 1)
              v[k] = __hip_atomic_load(lev + dep[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
          for (int k = 0; k < kLevDeps; ++k)
            if ((pending >> k & 1) && v[k] >= 0) {
              Lk = max(Lk, v[k] + 1);
              pending &= ~(1u << k);
            }
          L = Lk;
          ready = pending == 0;
        } else {
          for (int p = p0; p < p1; ++p) {
            const int v =
                __hip_atomic_load(lev + ci[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (v < 0) {
              ready = false;
              break;
            }
            L = max(L, v + 1);
          }
        }
        if (ready) {
          __hip_atomic_store(lev + i, L, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          done = true;
        } else if (wall_clock64() - t0 > limit ||
                   __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
          atomicOr(err, 2);
          done = true;
        }
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
}

// IKJ elimination of the rows of one level (rows k < i already final)
__global__ void k_ilu_rows(const int* rows, int r0, int r1, const int* rp, const int* ci,
                           const int* diag, double* lu, int* err) {
  int t = r0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= r1) return;
  int i = rows[t];
  int end = rp[i + 1];
  for (int p = rp[i]; p < diag[i]; ++p) {
    int k = ci[p];
    double lik = lu[p] / lu[diag[k]];
    lu[p] = lik;
    int a = p + 1, b = diag[k] + 1, bend = rp[k + 1];
    while (a < end && b < bend) {
      int ca = ci[a], cb = ci[b];
      if (ca == cb) {
        lu[a] = __builtin_fma(-lik, lu[b], lu[a]);  // one rounding, as in k_ilu_ranges
        ++a;
        ++b;
      } else if (ca < cb) {
        ++a;
      } else {
        ++b;
      }
    }
  }
  if (!(lu[diag[i]] > 0.0)) atomicOr(err, 1);
}

// ---- one-launch sweeps: level-ordered chunks with point-to-point waits ------
// Rows are taken in level order, in chunks that never straddle a level; a
// workgroup takes the next chunk from an atomic ticket, so the workgroup that
// holds the lowest unfinished ticket has every dependency (all in lower
// levels, hence earlier tickets) already written and always progresses.  A
// row waits only for its own dependencies: every output entry starts as a
// sentinel NaN and the value itself is the ready flag (device-coherent atomic
// 64/32-bit stores and loads, so no separate flag or fence is needed).  A wait
// is bounded: past the spin limit the kernel flags an error and moves on, so
// every wave always exits.
template <class T> struct Sentinel;
template <> struct Sentinel<double> {
  using U = unsigned long long;
  static constexpr U bits = 0x7FF4000000000BADull;
};
template <> struct Sentinel<float> {
  using U = unsigned int;
  static constexpr U bits = 0x7FA00BADu;
};

template <class T>
__device__ __forceinline__ void store_ready(T* p, T v) {
  using U = typename Sentinel<T>::U;
  U u;
  __builtin_memcpy(&u, &v, sizeof(T));
  if (u == Sentinel<T>::bits) u ^= 1;  // never publish the sentinel itself
  __hip_atomic_store(reinterpret_cast<U*>(p), u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class T>
__device__ __forceinline__ typename Sentinel<T>::U load_raw(const T* p) {
  using U = typename Sentinel<T>::U;
  return __hip_atomic_load(reinterpret_cast<const U*>(p), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until *p is published, given a first read u of it.  Polls back off up
// to ~0.4 us; the wait gives up after `limit` wall-clock ticks, or at once
// when another wait has given up (err != 0), so a broken dependency order
// ends the kernel quickly.  A wait that ends after more than limit / 2048
// ticks (about 1 ms) is counted in err[1]: waits that long mean the
// workgroups holding the dependencies were not running (another process's
// work on the device), the first sign before a wait runs out.
template <class T>
__device__ __forceinline__ T wait_ready(const T* p, typename Sentinel<T>::U u, int* err,
                                        unsigned long long limit) {
  using U = typename Sentinel<T>::U;
  const U* q = reinterpret_cast<const U*>(p);
  if (u == Sentinel<T>::bits) {
    const unsigned long long t0 = wall_clock64();
    int backoff = 1;
    while (u == Sentinel<T>::bits) {
      for (int k = 0; k < backoff; ++k) __builtin_amdgcn_s_sleep(1);
      backoff = backoff < 16 ? 2 * backoff : 16;
      u = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (u != Sentinel<T>::bits) {
        if (wall_clock64() - t0 > (limit >> 11)) atomicAdd(err + 1, 1);
        break;
      }
      if (wall_clock64() - t0 > limit ||
          __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        atomicOr(err, 2);
        u = 0;
        break;
      }
    }
  }
  T v;
  __builtin_memcpy(&v, &u, sizeof(T));
  return v;
}

// s -= sum_{p in [p0, p1)} lu[p] x[ci[p]], waiting for each x entry.  The
// reads of up to kDeps dependencies are issued together, so a row that finds
// them published pays one memory round trip, not one per dependency.
constexpr int kDeps = 8;

template <class T>
__device__ __forceinline__ void dot_ready(T& s, int p0, int p1, const int* ci, const T* lu,
                                          const T* x, int* err, unsigned long long limit) {
  using U = typename Sentinel<T>::U;
  for (int pb = p0; pb < p1; pb += kDeps) {
    U u[kDeps];
#pragma unroll
    for (int k = 0; k < kDeps; ++k)
      if (pb + k < p1) u[k] = load_raw<T>(x + ci[pb + k]);
#pragma unroll
    for (int k = 0; k < kDeps; ++k)
      if (pb + k < p1) s -= lu[pb + k] * wait_ready<T>(x + ci[pb + k], u[k], err, limit);
  }
}

template <class T>
__global__ void k_fill_sentinel(int n, T* x) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  using U = typename Sentinel<T>::U;
  if (i < n) reinterpret_cast<U*>(x)[i] = Sentinel<T>::bits;
}

// forward sweep y = L^{-1} b (unit L); also arms z (the backward sweep's
// output) with the sentinel
template <class T>
__global__ void __launch_bounds__(256)
k_sweep_lower(const int* rows, const int* chunk, int nchunks, const int* rp, const int* ci,
              const int* diag, const T* lu, const T* b, T* y, T* z, int* ticket, int* err,
              unsigned long long limit) {
  __shared__ int s_c;
  while (true) {
    if (threadIdx.x == 0) s_c = atomicAdd(ticket, 1);
    __syncthreads();
    const int c = s_c;
    __syncthreads();
    if (c >= nchunks) break;
    const int t = chunk[c] + threadIdx.x;
    if (t < chunk[c + 1]) {
      const int i = rows[t];
      T s = b[i];
      dot_ready<T>(s, rp[i], diag[i], ci, lu, y, err, limit);
      using U = typename Sentinel<T>::U;
      reinterpret_cast<U*>(z)[i] = Sentinel<T>::bits;
      store_ready<T>(y + i, s);
    }
  }
}

// backward sweep z = U^{-1} y
template <class T>
__global__ void __launch_bounds__(256)
k_sweep_upper(const int* rows, const int* chunk, int nchunks, const int* rp, const int* ci,
              const int* diag, const T* lu, const T* y, T* z, int* ticket, int* err,
              unsigned long long limit) {
  __shared__ int s_c;
  while (true) {
    if (threadIdx.x == 0) s_c = atomicAdd(ticket, 1);
    __syncthreads();
    const int c = s_c;
    __syncthreads();
    if (c >= nchunks) break;
    const int t = chunk[c] + threadIdx.x;
    if (t < chunk[c + 1]) {
      const int i = rows[t];
      T s = y[i];
      dot_ready<T>(s, diag[i] + 1, rp[i + 1], ci, lu, z, err, limit);
      store_ready<T>(z + i, s / lu[diag[i]]);
    }
  }
}

// Range sweeps.  A workgroup takes ranges in ticket order (ascending for the
// forward sweep, descending for the backward one) and walks a range level by
// level with a barrier between levels; values of rows inside the range are
// read from LDS, values of rows in earlier ranges are waited for in global
// memory, and every row is published there (value as ready flag) for the
// ranges after it.  While a level is computed, each thread already loads
// its row of the next level (ELL dependencies, factor values, and the first
// read of its dependencies outside the range), so the barrier, LDS reads
// and arithmetic are all that a level costs on the critical path.  A range
// depends only on earlier tickets, whose workgroups are already running, so
// the schedule always progresses; every wait is bounded as above.
template <class T>
struct SweepRow {
  using U = typename Sentinel<T>::U;
  int t, i, cnt;
  T in, dg;
  int col[kEll];
  T val[kEll];
  U raw[kEll];
};

// the part of a row's data addressed by its sweep position t alone (the
// input is gathered into sweep order beforehand)
// (loads are issued unconditionally -- position 0 stands in for "no row" --
// so every thread issues the same number of loads per level and the
// compiler's wait counts stay exact instead of draining all loads in flight)
template <class T>
__device__ __forceinline__ void fetch_static(SweepRow<T>& w, int t, const int* rows,
                                             const int* ecol, const T* eval, const int* ecnt,
                                             const T* ediag, const T* inp) {
  w.t = t;
  const int64_t u = t < 0 ? 0 : t;
  w.i = rows[u];
  w.cnt = ecnt[u];
  w.dg = ediag[u];
  w.in = inp[u];
#pragma unroll
  for (int k = 0; k < kEll; ++k) {
    w.col[k] = ecol[u * kEll + k];
    w.val[k] = eval[u * kEll + k];
  }
}

// first read of every dependency in global memory (only those outside the
// range [lo, hi) are used later; the others come from LDS)
template <class T>
__device__ __forceinline__ void fetch_raw(SweepRow<T>& w, const T* g) {
#pragma unroll
  for (int k = 0; k < kEll; ++k) w.raw[k] = load_raw<T>(g + max(w.col[k], 0));
}

template <class T, bool kUpper>
__device__ __forceinline__ void sweep_row(const SweepRow<T>& w, int lo, int hi, T* loc, T* g,
                                          T* arm, const int* ep0, const int* ci, const T* lu,
                                          int* err, unsigned long long limit) {
  using U = typename Sentinel<T>::U;
  T s = w.in;
#pragma unroll
  for (int k = 0; k < kEll; ++k) {
    const int j = w.col[k];
    if (j >= 0) {
      T v;
      if (j >= lo && j < hi) v = loc[j - lo];
      else v = wait_ready<T>(g + j, w.raw[k], err, limit);
      s -= w.val[k] * v;
    }
  }
  if (w.cnt > kEll) {  // dependencies past the ELL width, from the CSR
    const int p0 = ep0[w.t];
    for (int p = p0 + kEll; p < p0 + w.cnt; ++p) {
      const int j = ci[p];
      T v;
      if (j >= lo && j < hi) v = loc[j - lo];
      else v = wait_ready<T>(g + j, load_raw<T>(g + j), err, limit);
      s -= lu[p] * v;
    }
  }
  if constexpr (kUpper) s = s / w.dg;
  else reinterpret_cast<U*>(arm)[w.i] = Sentinel<T>::bits;
  loc[w.i - lo] = s;
  store_ready<T>(g + w.i, s);
}

// Range sweep kernel.  Each thread keeps four levels in flight in a register
// ring: at level k it issues the position-addressed loads of level k+3 and
// the outside-range reads of level k+2, then computes its row of level k
// (loads are issued ~3 levels before use, so a level costs about a barrier
// and its arithmetic).  The level loop is unrolled by four so the ring is
// indexed at compile time.
template <class T, bool kUpper>
__global__ void __launch_bounds__(256)
k_sweep_ranges(int n, int S, int nranges, const int* rows, const int* seg, const int* segbase,
               const int* ecol, const T* eval, const int* ecnt, const int* ep0, const T* ediag,
               const int* ci, const T* lu, const T* inp, T* out, T* arm, int* ticket, int* err,
               unsigned long long limit) {
  // dynamic LDS: the range's values (S entries of T), then its level
  // boundaries (max_segs + 1 ints; always in LDS, so every read of them is
  // an LDS read and never waits on the global loads in flight)
  extern __shared__ double lds_raw[];
  T* loc = reinterpret_cast<T*>(lds_raw);
  int* s_seg = reinterpret_cast<int*>(loc + S);
  __shared__ int s_c;
  const int tid = threadIdx.x, nt = blockDim.x;
  while (true) {
    if (tid == 0) s_c = atomicAdd(ticket, 1);
    __syncthreads();
    const int c = s_c;
    if (c >= nranges) break;
    const int r = kUpper ? nranges - 1 - c : c;
    const int r0 = r * S, r1 = min(n, r0 + S);
    const int sb = segbase[r], ns = segbase[r + 1] - sb;
    for (int k = tid; k <= ns; k += nt) s_seg[k] = seg[sb + k];
    __syncthreads();
    auto segat = [&](int k) { return s_seg[k]; };
    auto pos = [&](int lvl) {
      if (lvl >= ns) return -1;
      const int t = segat(lvl) + tid;
      return t < segat(lvl + 1) ? t : -1;
    };
    auto fst = [&](SweepRow<T>& w, int lvl) {
      fetch_static<T>(w, pos(lvl), rows, ecol, eval, ecnt, ediag, inp);
    };
    auto step = [&](int lvl, SweepRow<T>& cur, SweepRow<T>& n2, SweepRow<T>& n3) {
      fst(n3, lvl + 3);
      fetch_raw<T>(n2, out);
      if (cur.t >= 0) sweep_row<T, kUpper>(cur, r0, r1, loc, out, arm, ep0, ci, lu, err, limit);
      const int a = segat(lvl), b = segat(lvl + 1);
      for (int t = a + tid + nt; t < b; t += nt) {  // levels wider than the workgroup
        SweepRow<T> w;
        fetch_static<T>(w, t, rows, ecol, eval, ecnt, ediag, inp);
        fetch_raw<T>(w, out);
        sweep_row<T, kUpper>(w, r0, r1, loc, out, arm, ep0, ci, lu, err, limit);
      }
      lds_barrier();  // the level's values in loc; global traffic stays in flight
    };
    SweepRow<T> s0, s1, s2, s3;
    fst(s0, 0);
    fst(s1, 1);
    fst(s2, 2);
    fetch_raw<T>(s0, out);
    fetch_raw<T>(s1, out);
    for (int k = 0; k < ns; k += 4) {
      step(k, s0, s2, s3);
      if (k + 1 < ns) step(k + 1, s1, s3, s0);
      if (k + 2 < ns) step(k + 2, s2, s0, s1);
      if (k + 3 < ns) step(k + 3, s3, s1, s2);
    }
  }
}

// ILU(0) factorisation in one launch on the lower sweep's range schedule
// (the factorisation of row i needs exactly the rows its lower triangle
// refers to).  A workgroup takes ranges in ticket order and walks a range
// level by level with a barrier between levels.  Other rows read only the
// upper part of a pivot row (its diagonal and the entries right of it), so
// that part is published entry by entry with the value itself as the ready
// flag, as in the sweeps: every upper entry of lu starts as the sentinel
// (k_upper_arm), a finished entry is written with a device-coherent atomic
// store, and a reader waits on the entries it uses.  No fence is needed (an
// agent-scope fence writes back or invalidates a whole L2), and a wait is
// bounded as in the sweeps.  The lower part (the multipliers) is private to
// its row and written with plain stores.
__global__ void k_upper_arm(int n, const int* rp, const int* diag, double* lu) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    using U = Sentinel<double>::U;
    const int end = rp[i + 1];
    for (int p = diag[i]; p < end; ++p) reinterpret_cast<U*>(lu)[p] = Sentinel<double>::bits;
  }
}

__device__ __forceinline__ double ready_at(const double* lu, int p, int* werr,
                                           unsigned long long limit) {
  return wait_ready<double>(lu + p, load_raw<double>(lu + p), werr, limit);
}

// Row i entry by entry (rows wider than the staged form holds).  The lower
// part is eliminated in place, pivot by pivot; then each upper entry takes,
// in pivot order, the update of every pivot row that holds its column, and
// is published.  Each entry sees the same fused multiply-adds in the same
// order as in the IKJ merge.
__device__ void ilu_row_entries(int i, const int* rp, const int* ci, const int* diag,
                                const double* a, double* lu, int* err, int* werr,
                                unsigned long long limit) {
  const int p0 = rp[i], end = rp[i + 1], di = diag[i];
  for (int p = p0; p < di; ++p) {
    const int k = ci[p], dk = diag[k], bend = rp[k + 1];
    const double lik = lu[p] / ready_at(lu, dk, werr, limit);
    lu[p] = lik;
    int q = p + 1;
    for (int b = dk + 1; b < bend && q < di; ++b) {
      while (q < di && ci[q] < ci[b]) ++q;
      if (q < di && ci[q] == ci[b]) {
        lu[q] = __builtin_fma(-lik, ready_at(lu, b, werr, limit), lu[q]);
        ++q;
      }
    }
  }
  for (int q = di; q < end; ++q) {
    const int c = ci[q];
    double v = a[q];
    for (int p = p0; p < di; ++p) {
      const int k = ci[p], bend = rp[k + 1];
      for (int b = diag[k] + 1; b < bend && ci[b] <= c; ++b)
        if (ci[b] == c) v = __builtin_fma(-lu[p], ready_at(lu, b, werr, limit), v);
    }
    if (q == di && !(v > 0.0)) atomicOr(err, 1);
    store_ready<double>(lu + q, v);
  }
}

// Static data of one position of the lower schedule (the row, its values
// and the pivot entries its elimination reads), column-major over the n
// positions so that a wavefront's loads of one field are consecutive.  The
// pivot entries of a row are listed pivot by pivot: the pivot's diagonal
// (target kTgtDiag), then each entry of the pivot's upper part whose column
// the row holds, with the row slot it updates.  meta packs the row length,
// the number of pivots and the number of listed entries (kEntryPath: the
// row is too wide for the record and is taken entry by entry).
constexpr int kIluThreads = 128;  // threads of the factorisation workgroup
constexpr int kIluRowW = 16;      // row entries a record holds
constexpr int kIluDyn = 20;       // pivot entries a record lists
constexpr int kTgtDiag = 255;
constexpr int kEntryPath = 255;

struct IluRecs {
  int* row;
  int* p0;
  int* meta;
  double* av;
  int* pos;
  unsigned char* tgt;
};

__global__ void k_ilu_symbolic(int n, const int* rows, const int* rp, const int* ci,
                               const int* diag, const double* a, int stage_w, IluRecs R) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int i = rows[t], p0 = rp[i], len = rp[i + 1] - p0, nlow = diag[i] - p0;
  const int64_t N = n;
  int nd = 0;
  bool fits = len <= stage_w;
  for (int m = 0; m < nlow && fits; ++m) {
    const int k = ci[p0 + m], dk = diag[k], bend = rp[k + 1];
    if (nd == kIluDyn) {
      fits = false;
      break;
    }
    R.pos[nd * N + t] = dk;
    R.tgt[nd * N + t] = kTgtDiag;
    ++nd;
    int q = m + 1;
    for (int b = dk + 1; b < bend && q < len; ++b) {
      while (q < len && ci[p0 + q] < ci[b]) ++q;
      if (q < len && ci[p0 + q] == ci[b]) {
        if (nd == kIluDyn) {
          fits = false;
          break;
        }
        R.pos[nd * N + t] = b;
        R.tgt[nd * N + t] = static_cast<unsigned char>(q);
        ++nd;
        ++q;
      }
    }
  }
  R.row[t] = i;
  R.p0[t] = p0;
  R.meta[t] = fits ? len | nlow << 8 | nd << 16 : kEntryPath << 16;
  if (fits)
    for (int q = 0; q < len; ++q) R.av[q * N + t] = a[p0 + q];
}

struct IluCur {
  int row, p0, meta;
  double av[kIluRowW];
  int pos[kIluDyn];
  unsigned char tgt[kIluDyn];
};

// a position's record (all fields, so the loads need nothing but t); t < 0:
// no row
__device__ __forceinline__ void ilu_fetch(IluCur& c, int t, int n, const IluRecs& R) {
  c.meta = -1;
  if (t < 0) return;
  const int64_t N = n;
  c.row = R.row[t];
  c.p0 = R.p0[t];
  c.meta = R.meta[t];
#pragma unroll
  for (int q = 0; q < kIluRowW; ++q) c.av[q] = R.av[q * N + t];
#pragma unroll
  for (int j = 0; j < kIluDyn; ++j) {
    c.pos[j] = R.pos[j * N + t];
    c.tgt[j] = R.tgt[j * N + t];
  }
}

// Staged elimination of one row from its record: the listed pivot entries
// are read together (one round trip once they are published), then applied
// in list order, which is the order of the IKJ merge.  The row's values sit
// in the thread's LDS slots (`val`, slot q of this thread).
template <class Val>
__device__ __forceinline__ void ilu_staged(const IluCur& c, Val val, const int* rp,
                                           const int* ci, const int* diag, const double* a,
                                           double* lu, int* err, int* werr,
                                           unsigned long long limit) {
  if (c.meta < 0) return;
  const int nd = c.meta >> 16;
  if (nd == kEntryPath) {
    ilu_row_entries(c.row, rp, ci, diag, a, lu, err, werr, limit);
    return;
  }
  const int len = c.meta & 0xFF, nlow = (c.meta >> 8) & 0xFF;
  using U = Sentinel<double>::U;
  U raw[kIluDyn];
#pragma unroll
  for (int j = 0; j < kIluDyn; ++j)
    if (j < nd) raw[j] = load_raw<double>(lu + c.pos[j]);
#pragma unroll
  for (int q = 0; q < kIluRowW; ++q)
    if (q < len) val(q) = c.av[q];
  int m = 0;
  double lik = 0.0;
#pragma unroll
  for (int j = 0; j < kIluDyn; ++j)
    if (j < nd) {
      const double u = wait_ready<double>(lu + c.pos[j], raw[j], werr, limit);
      if (c.tgt[j] == kTgtDiag) {
        lik = val(m) / u;
        val(m) = lik;
        ++m;
      } else {
        val(c.tgt[j]) = __builtin_fma(-lik, u, val(c.tgt[j]));
      }
    }
  if (!(val(nlow) > 0.0)) atomicOr(err, 1);
#pragma unroll
  for (int q = 0; q < kIluRowW; ++q)
    if (q < len) {
      if (q < nlow) lu[c.p0 + q] = val(q);
      else store_ready<double>(lu + c.p0 + q, val(q));
    }
}

// The factorisation kernel: while a level's pivot entries are in flight,
// the records of the thread's row of the next level are loaded, so a level
// costs about one round trip on published values, its arithmetic and a
// barrier.  Dynamic LDS: the range's level boundaries (max_segs + 1 ints).
__global__ void __launch_bounds__(kIluThreads)
k_ilu_ranges(int n, int nranges, const int* seg, const int* segbase, IluRecs R, const int* rp,
             const int* ci, const int* diag, const double* a, double* lu, int* ticket, int* err,
             int* werr, unsigned long long limit) {
  extern __shared__ int s_seg[];
  __shared__ double s_val[kIluRowW * kIluThreads];
  __shared__ int s_c;
  const int tid = threadIdx.x;
  auto val = [&](int q) -> double& { return s_val[q * kIluThreads + tid]; };
  while (true) {
    if (tid == 0) s_c = atomicAdd(ticket, 1);
    __syncthreads();
    const int c = s_c;
    if (c >= nranges) break;
    const int sb = segbase[c], ns = segbase[c + 1] - sb;
    for (int k = tid; k <= ns; k += kIluThreads) s_seg[k] = seg[sb + k];
    __syncthreads();
    auto first = [&](int lvl) {
      if (lvl >= ns) return -1;
      const int t = s_seg[lvl] + tid;
      return t < s_seg[lvl + 1] ? t : -1;
    };
    IluCur cur, nxt;
    ilu_fetch(cur, first(0), n, R);
    for (int lvl = 0; lvl < ns; ++lvl) {
      ilu_fetch(nxt, first(lvl + 1), n, R);
      ilu_staged(cur, val, rp, ci, diag, a, lu, err, werr, limit);
      for (int t = s_seg[lvl] + tid + kIluThreads; t < s_seg[lvl + 1]; t += kIluThreads) {
        ilu_fetch(cur, t, n, R);  // levels wider than the workgroup
        ilu_staged(cur, val, rp, ci, diag, a, lu, err, werr, limit);
      }
      __syncthreads();  // a level's rows published before the next level waits on them
      cur = nxt;
    }
  }
}

// x[t] = v[rows[t]]: a sweep's input in sweep order
template <class T>
__global__ void k_gather(int n, const int* rows, const T* v, T* x) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) x[t] = v[rows[t]];
}

// ELL form of the dependencies of every position of a range schedule
__global__ void k_ell_build(int n, int upper, const int* rows, const int* rp, const int* diag,
                            const int* ci, int* ecol, int* epos, int* ecnt, int* ep0) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int i = rows[t];
  const int p0 = upper ? diag[i] + 1 : rp[i];
  const int p1 = upper ? rp[i + 1] : diag[i];
  ecnt[t] = p1 - p0;
  ep0[t] = p0;
  for (int k = 0; k < kEll; ++k) {
    const bool in = p0 + k < p1;
    ecol[static_cast<int64_t>(t) * kEll + k] = in ? ci[p0 + k] : -1;
    epos[static_cast<int64_t>(t) * kEll + k] = in ? p0 + k : -1;
  }
}

template <class T>
__global__ void k_ell_vals(int n, const int* rows, const int* diag, const int* epos,
                           const T* lu, T* eval, T* ediag) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  for (int k = 0; k < kEll; ++k) {
    const int p = epos[static_cast<int64_t>(t) * kEll + k];
    eval[static_cast<int64_t>(t) * kEll + k] = p >= 0 ? lu[p] : T(0);
  }
  ediag[t] = lu[diag[rows[t]]];
}

}  // namespace

// bound of one dataflow wait: 2 s of the device's constant-rate clock
unsigned long long wait_limit(Handle* h) {
  if (!h->wait_ticks) {
    int dev = 0, khz = 0;
    HIPX(hipGetDevice(&dev));
    HIPX(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    h->wait_ticks = 2000ull * static_cast<unsigned long long>(khz > 0 ? khz : 100000);
  }
  return h->wait_ticks;
}

namespace {

// dependency levels of both triangles: the two dataflow launches run side by
// side (they share nothing), then each level array is sorted into a schedule
void levels_both(Handle* h, Levels* outs[2], std::vector<int>* host_levs[2]) {
  const int n = h->n;
  unsigned g = blocks_for(n, kT);
  DBuf<int> lev[2] = {DBuf<int>(&h->alloc, n), DBuf<int>(&h->alloc, n)};
  DBuf<int> flags(&h->alloc, 4);  // per triangle: ticket, error
  for (int u = 0; u < 2; ++u)
    HIPX(hipMemsetAsync(lev[u], 0xFF, n * sizeof(int), h->stream));  // -1: not known yet
  HIPX(hipMemsetAsync(flags, 0, 4 * sizeof(int), h->stream));
  const int groups = std::min<int>((n + 255) / 256, 1024);
  {
    Fork fork(h);
    hipStream_t s0 = fork.next(), s1 = fork.next();
    LAUNCH_ON(h, s0, "ilu_levels", k_levels_df<false>, groups, 256, 0, n, h->rp.get(),
              h->ci.get(), h->diag.get(), lev[0].get(), flags.get(), flags.get() + 1,
              wait_limit(h));
    LAUNCH_ON(h, s1, "ilu_levels", k_levels_df<true>, groups, 256, 0, n, h->rp.get(),
              h->ci.get(), h->diag.get(), lev[1].get(), flags.get() + 2, flags.get() + 3,
              wait_limit(h));
    fork.join();
  }
  int hf[4] = {0, 0, 0, 0};
  HIPX(hipMemcpyAsync(hf, flags.get(), sizeof(hf), hipMemcpyDeviceToHost, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  FAMS_REQUIRE(hf[1] == 0 && hf[3] == 0, FAMS_ERR_DEVICE, "ILU level computation did not complete");
  for (int u = 0; u < 2; ++u) {
    Levels* out = outs[u];
    DBuf<int> iota(&h->alloc, n), keys(&h->alloc, n);
    out->rows.reset(&h->alloc, n);
    LAUNCH(h, "iota", k_iota, g, kT, 0, n, iota.get());
    int maxlev = 0;
    {
      std::vector<int>& hl = *host_levs[u];
      hl.resize(n);
      HIPX(hipMemcpyAsync(hl.data(), lev[u].get(), n * sizeof(int), hipMemcpyDeviceToHost,
                          h->stream));
      HIPX(hipStreamSynchronize(h->stream));
      for (int v : hl) maxlev = std::max(maxlev, v);
    }
    int bits = 1;
    while ((1 << bits) <= maxlev) ++bits;
    sort_pairs_i32(h, lev[u], keys, iota, out->rows, n, bits);
    DBuf<int> ptr(&h->alloc, maxlev + 2);
    LAUNCH(h, "level_ptr", k_level_ptr, g, kT, 0, n, keys.get(), ptr.get());
    out->ptr.assign(maxlev + 2, 0);
    HIPX(hipMemcpyAsync(out->ptr.data(), ptr.get(), (maxlev + 2) * sizeof(int),
                        hipMemcpyDeviceToHost, h->stream));
    HIPX(hipStreamSynchronize(h->stream));
  }
}

__global__ void k_d2f_ilu(int64_t n, const double* a, float* b) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) b[i] = static_cast<float>(a[i]);
}

// rows per range of the range sweeps: FAMS_ILU_RANGE (0 selects the
// level-chunk sweeps), default 8192
// widest row the factorisation stages in LDS (0: every row entry by entry)
int ilu_stage_width() {
  int w = kIluRowW;
  if (const char* e = std::getenv("FAMS_ILU_STAGE")) w = std::atoi(e);
  return std::max(0, std::min(w, kIluRowW));
}

int sweep_range_rows(Handle* h) {
  (void)h;
  int S = 8192;
  if (const char* e = std::getenv("FAMS_ILU_RANGE")) S = std::atoi(e);
  if (S < 0) S = 0;
  return std::min(S, 16384);
}

// range schedule of one sweep from the rows' global dependency levels: inside
// a range, rows of equal level are independent and every dependency inside
// the range has a lower level, so a workgroup can take the range level by
// level with a barrier between levels (counting sort per range, host side)
void range_table(Handle* h, const std::vector<int>& lev, int S, int upper, Ranges* R) {
  const int n = h->n;
  const int nr = (n + S - 1) / S;
  std::vector<int> rows(n), seg, segbase(nr + 1);
  std::vector<int> cnt;
  for (int r = 0; r < nr; ++r) {
    const int r0 = r * S, r1 = std::min(n, r0 + S);
    int lo = INT32_MAX, hi = 0;
    for (int i = r0; i < r1; ++i) {
      lo = std::min(lo, lev[i]);
      hi = std::max(hi, lev[i]);
    }
    cnt.assign(hi - lo + 2, 0);
    for (int i = r0; i < r1; ++i) ++cnt[lev[i] - lo + 1];
    for (size_t k = 1; k < cnt.size(); ++k) cnt[k] += cnt[k - 1];
    segbase[r] = static_cast<int>(seg.size());
    for (int L = 0; L <= hi - lo; ++L)
      if (cnt[L + 1] > cnt[L]) seg.push_back(r0 + cnt[L]);
    for (int i = r0; i < r1; ++i) rows[r0 + cnt[lev[i] - lo]++] = i;
  }
  segbase[nr] = static_cast<int>(seg.size());
  seg.push_back(n);
  R->max_segs = 0;
  for (int r = 0; r < nr; ++r) R->max_segs = std::max(R->max_segs, segbase[r + 1] - segbase[r]);
  R->S = S;
  R->nranges = nr;
  R->rows.reset(&h->alloc, n);
  R->seg.reset(&h->alloc, seg.size());
  R->segbase.reset(&h->alloc, nr + 1);
  HIPX(hipMemcpyAsync(R->rows, rows.data(), n * sizeof(int), hipMemcpyHostToDevice, h->stream));
  HIPX(hipMemcpyAsync(R->seg, seg.data(), seg.size() * sizeof(int), hipMemcpyHostToDevice,
                      h->stream));
  HIPX(hipMemcpyAsync(R->segbase, segbase.data(), (nr + 1) * sizeof(int), hipMemcpyHostToDevice,
                      h->stream));
  const size_t ne = static_cast<size_t>(n) * kEll;
  R->ecol.reset(&h->alloc, ne);
  R->epos.reset(&h->alloc, ne);
  R->ecnt.reset(&h->alloc, n);
  R->ep0.reset(&h->alloc, n);
  LAUNCH(h, "ilu_ell", k_ell_build, blocks_for(n, kT), kT, 0, n, upper, R->rows.get(),
         h->rp.get(), h->diag.get(), h->ci.get(), R->ecol.get(), R->epos.get(), R->ecnt.get(),
         R->ep0.get());
  R->eval64.free();  // the ELL values follow the factors: taken again on the next sweep
  R->ediag64.free();
  R->eval32.free();
  R->ediag32.free();
  HIPX(hipStreamSynchronize(h->stream));
}

// factor values of a range schedule in precision T (gathered once)
template <class T>
void ell_values(Handle* h, Ranges* R, const T* lu, DBuf<T>& ev, DBuf<T>& ed) {
  if (ev.get()) return;
  const int n = h->n;
  ev.reset(&h->alloc, static_cast<size_t>(n) * kEll);
  ed.reset(&h->alloc, n);
  LAUNCH(h, "ilu_ell", k_ell_vals<T>, blocks_for(n, kT), kT, 0, n, R->rows.get(),
         h->diag.get(), R->epos.get(), lu, ev.get(), ed.get());
}

// chunks of at most 256 rows inside one level
void chunk_table(Handle* h, Levels* L) {
  std::vector<int> cb;
  for (int l = 0; l < L->count(); ++l)
    for (int s = L->ptr[l]; s < L->ptr[l + 1]; s += 256) cb.push_back(s);
  cb.push_back(L->ptr.empty() ? 0 : L->ptr.back());
  L->nchunks = static_cast<int>(cb.size()) - 1;
  L->chunk.reset(&h->alloc, cb.size());
  HIPX(hipMemcpyAsync(L->chunk, cb.data(), cb.size() * sizeof(int), hipMemcpyHostToDevice,
                      h->stream));
  HIPX(hipStreamSynchronize(h->stream));
}

}  // namespace

void build_ilu(Handle* h) {
  const int n = h->n;
  DBuf<int> err(&h->alloc, 1);
  HIPX(hipMemsetAsync(err, 0, sizeof(int), h->stream));
  h->diag.reset(&h->alloc, n);
  LAUNCH(h, "diag_pos", k_diag_pos, blocks_for(n, kT), kT, 0, n, h->rp.get(), h->ci.get(),
         h->diag.get(), err.get());
  int e = 0;
  HIPX(hipMemcpyAsync(&e, err.get(), sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  FAMS_REQUIRE(e == 0, FAMS_ERR_INVALID_ARG, "a row of A has no stored diagonal");
  if (!h->smoother) return;
  PhaseTimer pt(h->stream);
  std::vector<int> lev_lo, lev_up;
  {
    Levels* outs[2] = {&h->lvl_lo, &h->lvl_up};
    std::vector<int>* hls[2] = {&lev_lo, &lev_up};
    levels_both(h, outs, hls);
  }
  pt.mark("ilu levels");
  chunk_table(h, &h->lvl_lo);
  chunk_table(h, &h->lvl_up);
  if (const int S = sweep_range_rows(h)) {
    range_table(h, lev_lo, S, 0, &h->rng_lo);
    range_table(h, lev_up, S, 1, &h->rng_up);
  }
  pt.mark("ilu schedules");
  h->info.ilu_levels_lower = h->lvl_lo.count();
  h->info.ilu_levels_upper = h->lvl_up.count();
  h->ilu.reset(&h->alloc, h->nnz);
  HIPX(hipMemcpyAsync(h->ilu, h->val.get(), h->nnz * sizeof(double), hipMemcpyDeviceToDevice,
                      h->stream));
  if (h->rng_lo.nranges > 0) {  // one launch on the range schedule
    const Ranges& L = h->rng_lo;
    DBuf<int> ticket(&h->alloc, 2);  // the ticket, then the wait error word
    HIPX(hipMemsetAsync(ticket, 0, 2 * sizeof(int), h->stream));
    // records of the lower schedule's positions
    DBuf<int> ri(&h->alloc, static_cast<size_t>(n) * (3 + kIluDyn));
    DBuf<double> rav(&h->alloc, static_cast<size_t>(n) * kIluRowW);
    DBuf<unsigned char> rtg(&h->alloc, static_cast<size_t>(n) * kIluDyn);
    const IluRecs R{ri.get(), ri.get() + n, ri.get() + 2 * static_cast<size_t>(n), rav.get(),
                    ri.get() + 3 * static_cast<size_t>(n), rtg.get()};
    LAUNCH(h, "ilu_factor", k_ilu_symbolic, blocks_for(n, kT), kT, 0, n, L.rows.get(),
           h->rp.get(), h->ci.get(), h->diag.get(), h->val.get(), ilu_stage_width(), R);
    LAUNCH(h, "ilu_factor", k_upper_arm, blocks_for(n, kT), kT, 0, n, h->rp.get(),
           h->diag.get(), h->ilu.get());
    const size_t lds = static_cast<size_t>(L.max_segs + 1) * sizeof(int);
    FAMS_REQUIRE(lds + sizeof(double) * kIluRowW * kIluThreads <=
                     static_cast<size_t>(lds_hw_budget(h)),
                 FAMS_ERR_CAPACITY, "ILU range schedule does not fit in LDS");
    allow_lds(reinterpret_cast<const void*>(&k_ilu_ranges), lds);
    LAUNCH(h, "ilu_factor", k_ilu_ranges, std::min(L.nranges, 2048), kIluThreads, lds, n,
           L.nranges, L.seg.get(), L.segbase.get(), R, h->rp.get(), h->ci.get(), h->diag.get(),
           h->val.get(), h->ilu.get(), ticket.get(), err.get(), ticket.get() + 1,
           wait_limit(h));
    int we = 0;
    HIPX(hipMemcpyAsync(&e, err.get(), sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPX(hipMemcpyAsync(&we, ticket.get() + 1, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPX(hipStreamSynchronize(h->stream));
    FAMS_REQUIRE(e != 0 || we == 0, FAMS_ERR_DEVICE,
                 "ILU(0) factorisation: a dependency wait exceeded its bound");
  } else {
    for (int L = 0; L < h->lvl_lo.count(); ++L) {
      int r0 = h->lvl_lo.ptr[L], r1 = h->lvl_lo.ptr[L + 1];
      LAUNCH(h, "ilu_factor", k_ilu_rows, blocks_for(r1 - r0, kT), kT, 0, h->lvl_lo.rows.get(),
             r0, r1, h->rp.get(), h->ci.get(), h->diag.get(), h->ilu.get(), err.get());
    }
    HIPX(hipMemcpyAsync(&e, err.get(), sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPX(hipStreamSynchronize(h->stream));
  }
  FAMS_REQUIRE(e == 0, FAMS_ERR_ZERO_PIVOT_ILU, "non-positive ILU(0) pivot");
  pt.mark("ilu factor");
  if (h->precision == FAMS_PREC_MIXED) {
    h->ilu32.reset(&h->alloc, h->nnz);
    LAUNCH(h, "d2f", k_d2f_ilu, blocks_for(h->nnz, kT), kT, 0, h->nnz, h->ilu.get(),
           h->ilu32.get());
  }
  // everything the sweeps keep in the handle, allocated now so that applying
  // the smoother allocates nothing: work tickets, the wait error word, the
  // sweep-order input and the factor values in the schedules' ELL form
  if (!h->ilu_ticket.get()) h->ilu_ticket.reset(&h->alloc, kTicketInts);
  if (!h->sweep_err.get()) {
    h->sweep_err.reset(&h->alloc, 2);   // error bits, long waits
    HIPX(hipMemsetAsync(h->sweep_err, 0, 2 * sizeof(int), h->stream));
  }
  if (h->rng_lo.nranges > 0) {
    if (h->precision == FAMS_PREC_MIXED) {
      if (!h->sweep_in32.get()) h->sweep_in32.reset(&h->alloc, n);
      ell_values<float>(h, &h->rng_lo, h->ilu32.get(), h->rng_lo.eval32, h->rng_lo.ediag32);
      ell_values<float>(h, &h->rng_up, h->ilu32.get(), h->rng_up.eval32, h->rng_up.ediag32);
    } else {
      if (!h->sweep_in64.get()) h->sweep_in64.reset(&h->alloc, n);
      ell_values<double>(h, &h->rng_lo, h->ilu.get(), h->rng_lo.eval64, h->rng_lo.ediag64);
      ell_values<double>(h, &h->rng_up, h->ilu.get(), h->rng_up.eval64, h->rng_up.ediag64);
    }
  }
}

namespace {

// the couplings of the per-medium systems A^mm and A^ff (and, with wells,
// the wells' own diagonal): both ends in one medium (medium_of)
__global__ void k_media_count(int n, int nm, int nwb, const int* rp, const int* ci, int* cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  int c = 0;
  if (i < n) {
    const int mi = medium_of(i, nm, nwb);
    for (int p = rp[i]; p < rp[i + 1]; ++p) c += medium_of(ci[p], nm, nwb) == mi;
  }
  cnt[i] = c;
}

__global__ void k_media_fill(int n, int nm, int nwb, const int* rp, const int* ci,
                             const double* val, const int* nrp, int* nci, double* nval) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int mi = medium_of(i, nm, nwb);
  int o = nrp[i];
  for (int p = rp[i]; p < rp[i + 1]; ++p)
    if (medium_of(ci[p], nm, nwb) == mi) {
      nci[o] = ci[p];
      nval[o] = val[p];
      ++o;
    }
}

}  // namespace

// The extra smoothing stage on the per-medium sub-systems (Sec. 3.2: another
// smoothing stage with iterations on A^mm and A^ff): one ILU(0) application
// of diag(A^mm, A^ff), i.e. of A without the couplings between the media,
// whose factors and sweep schedules live in a handle of their own built by
// the same code as the main ILU(0).
void build_block_smoother(Handle* h) {
  const int n = h->n;
  std::unique_ptr<Handle> b(new Handle());
  b->stream = h->stream;
  b->alloc.stream = h->stream;
  b->alloc.hook = h->alloc.hook;
  b->alloc.has_hook = h->alloc.has_hook;
  b->prof.stream = h->stream;
  b->precision = h->precision;
  b->smoother = 1;
  b->n = n;
  b->nm = h->nm;
  b->nw = h->nw;
  const int nwb = n - h->nw;
  {
    DBuf<int> cnt(&b->alloc, n + 1);
    LAUNCH(h, "media_split", k_media_count, blocks_for(n + 1, kT), kT, 0, n, h->nm, nwb,
           h->rp.get(), h->ci.get(), cnt.get());
    b->rp.reset(&b->alloc, n + 1);
    exclusive_scan_i32(h, cnt, b->rp, n + 1);
    int nnz = 0;
    HIPX(hipMemcpyAsync(&nnz, b->rp.get() + n, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPX(hipStreamSynchronize(h->stream));
    b->nnz = nnz;
    b->ci.reset(&b->alloc, nnz);
    b->val.reset(&b->alloc, nnz);
    LAUNCH(h, "media_split", k_media_fill, blocks_for(n, kT), kT, 0, n, h->nm, nwb,
           h->rp.get(), h->ci.get(), h->val.get(), b->rp.get(), b->ci.get(), b->val.get());
  }
  build_ilu(b.get());
  if (h->precision == FAMS_PREC_MIXED) h->blk_x32.reset(&h->alloc, n);
  else h->blk_x.reset(&h->alloc, n);
  HIPX(hipStreamSynchronize(h->stream));
  h->blk = std::move(b);
}

// x = U^{-1} L^{-1} b.  `y` is scratch of n entries.
template <class T>
void ilu_apply(Handle* h, const T* lu, const T* b, T* x, T* y) {
  if (!h->ilu_ticket.get()) h->ilu_ticket.reset(&h->alloc, kTicketInts);
  if (!h->sweep_err.get()) {
    h->sweep_err.reset(&h->alloc, 2);   // error bits, long waits
    HIPX(hipMemsetAsync(h->sweep_err, 0, 2 * sizeof(int), h->stream));
  }
  HIPX(hipMemsetAsync(h->ilu_ticket, 0, 2 * sizeof(int), h->stream));
  const int n = h->n;
  LAUNCH(h, "ilu_arm", k_fill_sentinel<T>, blocks_for(n, kT), kT, 0, n, y);
  wait_limit(h);
  if (h->rng_lo.nranges > 0) {
    Ranges& L = h->rng_lo;
    Ranges& U = h->rng_up;
    const T *lv, *ld, *uv, *ud;
    if constexpr (std::is_same<T, double>::value) {
      ell_values<double>(h, &L, lu, L.eval64, L.ediag64);
      ell_values<double>(h, &U, lu, U.eval64, U.ediag64);
      lv = L.eval64.get(); ld = L.ediag64.get(); uv = U.eval64.get(); ud = U.ediag64.get();
    } else {
      ell_values<float>(h, &L, lu, L.eval32, L.ediag32);
      ell_values<float>(h, &U, lu, U.eval32, U.ediag32);
      lv = L.eval32.get(); ld = L.ediag32.get(); uv = U.eval32.get(); ud = U.ediag32.get();
    }
    const size_t lds = static_cast<size_t>(L.S) * sizeof(T) +
                       static_cast<size_t>(std::max(L.max_segs, U.max_segs) + 1) * sizeof(int);
    FAMS_REQUIRE(lds <= static_cast<size_t>(lds_hw_budget(h)), FAMS_ERR_CAPACITY,
                 "ILU range schedule does not fit in LDS");
    allow_lds(reinterpret_cast<const void*>(&k_sweep_ranges<T, false>), lds);
    allow_lds(reinterpret_cast<const void*>(&k_sweep_ranges<T, true>), lds);
    T* inp;
    if constexpr (std::is_same<T, double>::value) {
      if (!h->sweep_in64.get()) h->sweep_in64.reset(&h->alloc, n);
      inp = h->sweep_in64.get();
    } else {
      if (!h->sweep_in32.get()) h->sweep_in32.reset(&h->alloc, n);
      inp = h->sweep_in32.get();
    }
    LAUNCH(h, "ilu_gather", k_gather<T>, blocks_for(n, kT), kT, 0, n, L.rows.get(), b, inp);
    LAUNCH(h, "ilu_lower", (k_sweep_ranges<T, false>), std::min(L.nranges, 2048), 256, lds, n,
           L.S, L.nranges, L.rows.get(), L.seg.get(), L.segbase.get(), L.ecol.get(), lv,
           L.ecnt.get(), L.ep0.get(), ld, h->ci.get(), lu, inp, y, x, h->ilu_ticket.get(),
           h->sweep_err.get(), h->wait_ticks);
    LAUNCH(h, "ilu_gather", k_gather<T>, blocks_for(n, kT), kT, 0, n, U.rows.get(), y, inp);
    LAUNCH(h, "ilu_upper", (k_sweep_ranges<T, true>), std::min(U.nranges, 2048), 256, lds, n,
           U.S, U.nranges, U.rows.get(), U.seg.get(), U.segbase.get(), U.ecol.get(), uv,
           U.ecnt.get(), U.ep0.get(), ud, h->ci.get(), lu, inp, x, nullptr,
           h->ilu_ticket.get() + 1, h->sweep_err.get(), h->wait_ticks);
    return;
  }
  // a window of ~kSweepGroups chunks in flight: enough to overlap tens of
  // levels, few enough that waiting rows do not flood the memory system
  const int g_lo = std::min(h->lvl_lo.nchunks, kSweepGroups);
  const int g_up = std::min(h->lvl_up.nchunks, kSweepGroups);
  LAUNCH(h, "ilu_lower", k_sweep_lower<T>, g_lo, 256, 0, h->lvl_lo.rows.get(),
         h->lvl_lo.chunk.get(), h->lvl_lo.nchunks, h->rp.get(), h->ci.get(), h->diag.get(), lu,
         b, y, x, h->ilu_ticket.get(), h->sweep_err.get(), h->wait_ticks);
  LAUNCH(h, "ilu_upper", k_sweep_upper<T>, g_up, 256, 0, h->lvl_up.rows.get(),
         h->lvl_up.chunk.get(), h->lvl_up.nchunks, h->rp.get(), h->ci.get(), h->diag.get(), lu,
         y, x, h->ilu_ticket.get() + 1, h->sweep_err.get(), h->wait_ticks);
}

namespace {

// ---- sweeps of K right-hand sides in lock-step --------------------------------
// Vectors hold K values per row (x[i * K + r], r = right-hand side).  The
// schedule is the level order of the one-launch sweeps cut into chunks of at
// most kBlkRows rows inside one level; a workgroup of kBlkRows x K threads
// takes a chunk by ticket and gives each row K consecutive lanes, one per
// right-hand side.  The K lanes of a row read the row's factor entries at the
// same addresses (one transaction) and gather the K consecutive values of
// each dependency (one contiguous stretch); lane r waits only for entry r of
// the rows it depends on (value as ready flag, bounded waits).
//
// Chunks are handed out by ncls counters (one per XCD when the grid allows,
// kTicketStride ints apart): workgroup b draws chunk cls + ncls t, t from
// counter cls = b % ncls, so each class takes its chunks in increasing
// order and no counter serves every workgroup of the device.  Waits stay
// deadlock-free: the lowest chunk not yet drawn belongs to a class whose
// workgroups all hold lower chunks, which wait only on lower chunks still,
// so one of them finishes and draws it.
constexpr int kBlkRows = 64;
// rows per chunk for K lanes per row: workgroups of at most 1024 threads
template <int K>
constexpr int blk_rows() { return K <= 16 ? kBlkRows : 1024 / K; }

template <class T, bool kUpper, int K>
__global__ void __launch_bounds__(blk_rows<K>() * K)
k_bsweep(const int* rows, const int* chunk, int nchunks, const int* rp, const int* ci,
         const int* diag, const T* lu, const T* in, T* out, T* arm, const T* add, double* sum,
         int* ticket, int ncls, int* err, unsigned long long limit) {
  using U = typename Sentinel<T>::U;
  __shared__ int s_c;
  const int r = threadIdx.x % K, slot = threadIdx.x / K;
  const int cls = blockIdx.x % ncls;
  int* my = ticket + kTicketStride * cls;
  while (true) {
    if (threadIdx.x == 0) s_c = cls + ncls * atomicAdd(my, 1);
    __syncthreads();
    const int c = s_c;
    __syncthreads();
    if (c >= nchunks) break;
    const int t = chunk[c] + slot;
    if (t < chunk[c + 1]) {
      const int i = rows[t];
      const int dg = diag[i];
      const int p0 = kUpper ? dg + 1 : rp[i];
      const int p1 = kUpper ? rp[i + 1] : dg;
      const int64_t o = static_cast<int64_t>(i) * K + r;
      T s = in[o];
      // the addend is read with the row's input, off the dependency chain
      const T ad = (kUpper && sum) ? add[o] : T(0);
      for (int pb = p0; pb < p1; pb += kDeps) {
        U u[kDeps];
        int j[kDeps];
        T l[kDeps];
#pragma unroll
        for (int k = 0; k < kDeps; ++k)
          if (pb + k < p1) {
            j[k] = ci[pb + k];
            l[k] = lu[pb + k];
          }
#pragma unroll
        for (int k = 0; k < kDeps; ++k)
          if (pb + k < p1) u[k] = load_raw<T>(out + static_cast<int64_t>(j[k]) * K + r);
#pragma unroll
        for (int k = 0; k < kDeps; ++k)
          if (pb + k < p1)
            s -= l[k] * wait_ready<T>(out + static_cast<int64_t>(j[k]) * K + r, u[k], err, limit);
      }
      if constexpr (kUpper) {
        s = s / lu[dg];
      } else {
        reinterpret_cast<U*>(arm)[o] = Sentinel<T>::bits;
      }
      store_ready<T>(out + o, s);
      // the two-stage sum in FP64 once the row is published (sum = add + x)
      if (kUpper && sum) sum[o] = static_cast<double>(ad) + static_cast<double>(s);
    }
  }
}

template <class T>
__global__ void k_bfill_sentinel(int64_t n, T* x) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  using U = typename Sentinel<T>::U;
  if (i < n) reinterpret_cast<U*>(x)[i] = Sentinel<T>::bits;
}

// chunks of at most `rows` rows inside one level (the lock-step sweeps; 64
// rows, or 32 for groups of 32 right-hand sides), kept in the level structure
void block_chunk_table(Handle* h, Levels* L, int rows) {
  DBuf<int>& tab = rows == kBlkRows ? L->bchunk : L->bchunk32;
  int& count = rows == kBlkRows ? L->nbchunks : L->nbchunks32;
  if (tab.get()) return;
  std::vector<int> cb;
  for (int l = 0; l < L->count(); ++l)
    for (int s = L->ptr[l]; s < L->ptr[l + 1]; s += rows) cb.push_back(s);
  cb.push_back(L->ptr.empty() ? 0 : L->ptr.back());
  count = static_cast<int>(cb.size()) - 1;
  tab.reset(&h->alloc, cb.size());
  HIPX(hipMemcpyAsync(tab, cb.data(), cb.size() * sizeof(int), hipMemcpyHostToDevice,
                      h->stream));
  HIPX(hipStreamSynchronize(h->stream));
}

}  // namespace

// x = U^{-1} L^{-1} b for K right-hand sides in lock-step (x[i * K + r]);
// y is scratch of n * K entries; with `sum`, also sum = add + x in FP64
template <class T, int K>
void ilu_apply_block(Handle* h, const T* lu, const T* b, T* x, T* y, const T* add, double* sum) {
  if (!h->ilu_ticket.get()) h->ilu_ticket.reset(&h->alloc, kTicketInts);
  if (!h->sweep_err.get()) {
    h->sweep_err.reset(&h->alloc, 2);   // error bits, long waits
    HIPX(hipMemsetAsync(h->sweep_err, 0, 2 * sizeof(int), h->stream));
  }
  constexpr int rows = blk_rows<K>();
  block_chunk_table(h, &h->lvl_lo, rows);
  block_chunk_table(h, &h->lvl_up, rows);
  const int nlo = rows == kBlkRows ? h->lvl_lo.nbchunks : h->lvl_lo.nbchunks32;
  const int nup = rows == kBlkRows ? h->lvl_up.nbchunks : h->lvl_up.nbchunks32;
  const int* clo = rows == kBlkRows ? h->lvl_lo.bchunk.get() : h->lvl_lo.bchunk32.get();
  const int* cup = rows == kBlkRows ? h->lvl_up.bchunk.get() : h->lvl_up.bchunk32.get();
  int* tlo = h->ilu_ticket.get() + kTicketBlock;
  int* tup = tlo + kXcd * kTicketStride;
  HIPX(hipMemsetAsync(tlo, 0, 2 * kXcd * kTicketStride * sizeof(int), h->stream));
  const int64_t nk = static_cast<int64_t>(h->n) * K;
  LAUNCH(h, "bilu_arm", k_bfill_sentinel<T>, blocks_for(nk, kT), kT, 0, nk, y);
  const unsigned long long lim = wait_limit(h);
  // about 2048 threads per compute unit in flight
  const int cap = 256 * 2048 / (rows * K);
  const int groups_lo = std::min(nlo, cap);
  const int groups_up = std::min(nup, cap);
  LAUNCH(h, "bilu_lower", (k_bsweep<T, false, K>), groups_lo, rows * K, 0,
         h->lvl_lo.rows.get(), clo, nlo, h->rp.get(), h->ci.get(), h->diag.get(), lu, b, y, x,
         static_cast<const T*>(nullptr), static_cast<double*>(nullptr), tlo,
         std::min(groups_lo, kXcd), h->sweep_err.get(), lim);
  LAUNCH(h, "bilu_upper", (k_bsweep<T, true, K>), groups_up, rows * K, 0,
         h->lvl_up.rows.get(), cup, nup, h->rp.get(), h->ci.get(), h->diag.get(), lu,
         static_cast<const T*>(y), x, static_cast<T*>(nullptr), add, sum, tup,
         std::min(groups_up, kXcd), h->sweep_err.get(), lim);
}

#define FAMS_ILU_BLOCK(T, K) \
  template void ilu_apply_block<T, K>(Handle*, const T*, const T*, T*, T*, const T*, double*);
FAMS_ILU_BLOCK(double, 2)
FAMS_ILU_BLOCK(double, 4)
FAMS_ILU_BLOCK(double, 8)
FAMS_ILU_BLOCK(double, 16)
FAMS_ILU_BLOCK(double, 32)
FAMS_ILU_BLOCK(float, 2)
FAMS_ILU_BLOCK(float, 4)
FAMS_ILU_BLOCK(float, 8)
FAMS_ILU_BLOCK(float, 16)
FAMS_ILU_BLOCK(float, 32)
#undef FAMS_ILU_BLOCK

template void ilu_apply<double>(Handle*, const double*, const double*, double*, double*);
template void ilu_apply<float>(Handle*, const float*, const float*, float*, float*);

}  // namespace fams
