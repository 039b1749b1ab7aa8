// ILU(0) smoother of Table 1 step 7 (Sec. 3.2): incomplete LU of A on A's own
// sparsity pattern, rows in their given (natural) order, and its application
// x = U^{-1} L^{-1} b by level-scheduled triangular sweeps.
//
// Level of row i in the lower sweep = 1 + max level of the rows j < i it
// depends on (0 if none); the upper sweep uses j > i.  Rows of one level are
// independent, so each level is one launch with a thread per row; the
// natural ordering -- and hence the smoother itself -- is unchanged.
#include <algorithm>
#include <vector>

#include "internal.hpp"

namespace fams {
namespace {

constexpr int kT = 256;

__global__ void k_diag_pos(int n, const int* rp, const int* ci, int* diag, int* err) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int d = -1;
  for (int p = rp[i]; p < rp[i + 1]; ++p)
    if (ci[p] == i) d = p;
  diag[i] = d;
  if (d < 0) atomicOr(err, 1);
}

__global__ void k_level_relax(int n, const int* rp, const int* ci, const int* diag, int upper,
                              int* lev, int* changed) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int m = 0;
  int a = upper ? diag[i] + 1 : rp[i];
  int b = upper ? rp[i + 1] : diag[i];
  for (int p = a; p < b; ++p) m = max(m, lev[ci[p]] + 1);
  if (m > lev[i]) {
    lev[i] = m;
    *changed = 1;
  }
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
        lu[a] -= lik * lu[b];
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

template <class T>
__global__ void k_trsv_lower(const int* rows, int r0, int r1, const int* rp, const int* ci,
                             const int* diag, const T* lu, const T* b, T* x) {
  int t = r0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= r1) return;
  int i = rows[t];
  T s = b[i];
  for (int p = rp[i]; p < diag[i]; ++p) s -= lu[p] * x[ci[p]];
  x[i] = s;
}

template <class T>
__global__ void k_trsv_upper(const int* rows, int r0, int r1, const int* rp, const int* ci,
                             const int* diag, const T* lu, T* x) {
  int t = r0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= r1) return;
  int i = rows[t];
  T s = x[i];
  for (int p = diag[i] + 1; p < rp[i + 1]; ++p) s -= lu[p] * x[ci[p]];
  x[i] = s / lu[diag[i]];
}

void levels(Handle* h, int upper, Levels* out) {
  const int n = h->n;
  unsigned g = blocks_for(n, kT);
  DBuf<int> lev(&h->alloc, n), changed(&h->alloc, 1);
  HIPX(hipMemsetAsync(lev, 0, n * sizeof(int), h->stream));
  for (int it = 0;; ++it) {
    FAMS_REQUIRE(it < 1000000, FAMS_ERR_DEVICE, "ILU level computation did not converge");
    HIPX(hipMemsetAsync(changed, 0, sizeof(int), h->stream));
    for (int s = 0; s < 8; ++s)
      LAUNCH(h, "ilu_levels", k_level_relax, g, kT, 0, n, h->rp.get(), h->ci.get(),
             h->diag.get(), upper, lev.get(), changed.get());
    int c = 0;
    HIPX(hipMemcpyAsync(&c, changed.get(), sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPX(hipStreamSynchronize(h->stream));
    if (!c) break;
  }
  DBuf<int> iota(&h->alloc, n), keys(&h->alloc, n);
  out->rows.reset(&h->alloc, n);
  LAUNCH(h, "iota", k_iota, g, kT, 0, n, iota.get());
  int maxlev = 0;
  {
    std::vector<int> hl(n);
    HIPX(hipMemcpyAsync(hl.data(), lev.get(), n * sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPX(hipStreamSynchronize(h->stream));
    for (int v : hl) maxlev = std::max(maxlev, v);
  }
  int bits = 1;
  while ((1 << bits) <= maxlev) ++bits;
  sort_pairs_i32(h, lev, keys, iota, out->rows, n, bits);
  DBuf<int> ptr(&h->alloc, maxlev + 2);
  LAUNCH(h, "level_ptr", k_level_ptr, g, kT, 0, n, keys.get(), ptr.get());
  out->ptr.assign(maxlev + 2, 0);
  HIPX(hipMemcpyAsync(out->ptr.data(), ptr.get(), (maxlev + 2) * sizeof(int),
                      hipMemcpyDeviceToHost, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
}

__global__ void k_d2f_ilu(int64_t n, const double* a, float* b) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) b[i] = static_cast<float>(a[i]);
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
  levels(h, 0, &h->lvl_lo);
  levels(h, 1, &h->lvl_up);
  h->info.ilu_levels_lower = h->lvl_lo.count();
  h->info.ilu_levels_upper = h->lvl_up.count();
  h->ilu.reset(&h->alloc, h->nnz);
  HIPX(hipMemcpyAsync(h->ilu, h->val.get(), h->nnz * sizeof(double), hipMemcpyDeviceToDevice,
                      h->stream));
  for (int L = 0; L < h->lvl_lo.count(); ++L) {
    int r0 = h->lvl_lo.ptr[L], r1 = h->lvl_lo.ptr[L + 1];
    LAUNCH(h, "ilu_factor", k_ilu_rows, blocks_for(r1 - r0, kT), kT, 0, h->lvl_lo.rows.get(), r0,
           r1, h->rp.get(), h->ci.get(), h->diag.get(), h->ilu.get(), err.get());
  }
  HIPX(hipMemcpyAsync(&e, err.get(), sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  FAMS_REQUIRE(e == 0, FAMS_ERR_ZERO_PIVOT_ILU, "non-positive ILU(0) pivot");
  if (h->precision == FAMS_PREC_MIXED) {
    h->ilu32.reset(&h->alloc, h->nnz);
    LAUNCH(h, "d2f", k_d2f_ilu, blocks_for(h->nnz, kT), kT, 0, h->nnz, h->ilu.get(),
           h->ilu32.get());
  }
}

template <class T>
void ilu_apply(Handle* h, const T* lu, const T* b, T* x) {
  for (int L = 0; L < h->lvl_lo.count(); ++L) {
    int r0 = h->lvl_lo.ptr[L], r1 = h->lvl_lo.ptr[L + 1];
    LAUNCH(h, "ilu_lower", k_trsv_lower<T>, blocks_for(r1 - r0, kT), kT, 0,
           h->lvl_lo.rows.get(), r0, r1, h->rp.get(), h->ci.get(), h->diag.get(), lu, b, x);
  }
  for (int L = 0; L < h->lvl_up.count(); ++L) {
    int r0 = h->lvl_up.ptr[L], r1 = h->lvl_up.ptr[L + 1];
    LAUNCH(h, "ilu_upper", k_trsv_upper<T>, blocks_for(r1 - r0, kT), kT, 0,
           h->lvl_up.rows.get(), r0, r1, h->rp.get(), h->ci.get(), h->diag.get(), lu, x);
  }
}

template void ilu_apply<double>(Handle*, const double*, const double*, double*);
template void ilu_apply<float>(Handle*, const float*, const float*, float*);

}  // namespace fams
