// The F-AMS iteration (Table 1) on the GPU, as a Richardson loop or as the
// right preconditioner of restarted GMRES (Sec. 4.6).
//
// Stage (Table 1 steps 5-7) applied to a residual r:
//   r_c = R r;  x_c = A_c^{-1} r_c;  dp1 = P x_c;       (multiscale stage)
//   r_half = r - A dp1;  dp2 = U^{-1} L^{-1} r_half;    (ILU(0) smoothing)
//   z = dp1 + dp2.
// Precision form: the stage runs on FP32 copies of A, P, R and the ILU(0)
// factors with FP32 vectors; the coarse solve, the outer residual q - A p,
// the Krylov basis and the solution update stay FP64.  Because the FP32
// stage is not exactly linear, GMRES keeps the preconditioned vectors
// (flexible GMRES); with an FP64 stage this is the same iteration as
// right-preconditioned GMRES.
//
// Reductions are two-stage with a fixed block count and fixed order, so a
// solve is bitwise reproducible.
#include <chrono>
#include <cmath>
#include <type_traits>
#include <vector>

#include "internal.hpp"

namespace fams {
namespace {

constexpr int kT = 256;
constexpr int kRedBlocks = 512;

// y = b - A x (b may be null: y = -A x); 8 lanes per row, so a wavefront
// reads 8 consecutive rows' entries as one contiguous stretch; fixed-order
// shuffle reduction (deterministic).
constexpr int kSub = 8;
template <class TV, class TX, class TB, class TY>
__global__ void __launch_bounds__(256)
k_resid(int n, const int* rp, const int* ci, const TV* val, const TX* x, const TB* b, TY* y) {
  const int i = blockIdx.x * (blockDim.x / kSub) + threadIdx.x / kSub;
  const int l = threadIdx.x % kSub;
  double s = 0.0;
  if (i < n)
    for (int p = rp[i] + l; p < rp[i + 1]; p += kSub)
      s += static_cast<double>(val[p]) * static_cast<double>(x[ci[p]]);
  for (int o = kSub / 2; o > 0; o >>= 1) s += __shfl_down(s, o, kSub);
  if (i < n && l == 0) y[i] = static_cast<TY>((b ? static_cast<double>(b[i]) : 0.0) - s);
}

// y = M x with 8 lanes per row (see k_resid)
template <class TV, class TX, class TY>
__global__ void __launch_bounds__(256)
k_spmv8(int n, const int* rp, const int* ci, const TV* val, const TX* x, TY* y) {
  const int i = blockIdx.x * (blockDim.x / kSub) + threadIdx.x / kSub;
  const int l = threadIdx.x % kSub;
  double s = 0.0;
  if (i < n)
    for (int p = rp[i] + l; p < rp[i + 1]; p += kSub)
      s += static_cast<double>(val[p]) * static_cast<double>(x[ci[p]]);
  for (int o = kSub / 2; o > 0; o >>= 1) s += __shfl_down(s, o, kSub);
  if (i < n && l == 0) y[i] = static_cast<TY>(s);
}

// y[r] = sum_k M[r,k] x[k] for short fat rows (R = P^T has ~N/n_c entries per
// row): one wavefront per row, lanes stride over the row, fixed-order shuffle
// reduction -- deterministic.
template <class TV, class TX>
__global__ void __launch_bounds__(256)
k_spmv_wave(int nrows, const int* rp, const int* ci, const TV* val, const TX* x, double* y) {
  int row = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  int lane = threadIdx.x % 64;
  if (row >= nrows) return;
  double s = 0.0;
  for (int p = rp[row] + lane; p < rp[row + 1]; p += 64)
    s += static_cast<double>(val[p]) * static_cast<double>(x[ci[p]]);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (lane == 0) y[row] = s;
}

__device__ double block_sum(double v) {
  __shared__ double s[kT / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  int w = threadIdx.x / 64, l = threadIdx.x % 64;
  __syncthreads();
  if (l == 0) s[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x / 64); ++k) r += s[k];
  return r;
}

__global__ void k_dot_part(int64_t n, const double* a, const double* b, double* part) {
  double s = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    s += a[i] * b[i];
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out[k] (+)= sum over blocks of part[b * stride + k]: one workgroup per k,
// strided partial sums then a fixed tree -- deterministic
__global__ void __launch_bounds__(256)
k_reduce(int nblk, int nv, int stride, const double* part, double* out, int accumulate) {
  const int k = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += part[static_cast<int64_t>(b) * stride + k];
  s = block_sum(s);
  if (threadIdx.x == 0) out[k] = accumulate ? out[k] + s : s;
}

// part[b * stride + k] = sum over this block's rows of V_k . w, k < nv
__global__ void k_mdot_part(int64_t n, int nv, const double* V, int64_t ldv, const double* w,
                            double* part, int stride) {
  for (int k = 0; k < nv; ++k) {
    const double* v = V + k * ldv;
    double s = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
      s += v[i] * w[i];
    s = block_sum(s);
    if (threadIdx.x == 0) part[static_cast<int64_t>(blockIdx.x) * stride + k] = s;
    __syncthreads();
  }
}

// w -= sum_k coef[k] V_k   (or x += sum_k coef[k] V_k with sign = +1)
__global__ void k_maxpy(int64_t n, int nv, const double* V, int64_t ldv, const double* coef,
                        double sign, double* w) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < nv; ++k) s += coef[k] * V[k * ldv + i];
  w[i] += sign * s;
}

__global__ void k_scale_by(int64_t n, const double* x, const double* den, double* y) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i] / *den;
}

__global__ void k_axpy(int64_t n, double a, const double* x, double* y) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

template <class TA, class TB, class TY>
__global__ void k_add(int64_t n, const TA* a, const TB* b, TY* y) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = static_cast<TY>(static_cast<double>(a[i]) + static_cast<double>(b[i]));
}

template <class TA, class TY>
__global__ void k_cast(int64_t n, const TA* a, TY* y) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = static_cast<TY>(a[i]);
}

__global__ void k_fill(int64_t n, double v, double* y) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = v;
}

__global__ void k_vadd(int nv, const double* b, double* a) {
  int k = threadIdx.x;
  if (k < nv) a[k] += b[k];
}

__global__ void k_sqrt_into(const double* src, double* dst) { *dst = sqrt(*src); }

// GMRES small dense part (one thread): Hessenberg column j from hcol,
// previous rotations, the new rotation and the residual estimate
struct GmresState {
  double* H;    // (m+1) x m, column-major
  double* cs;   // m
  double* sn;   // m
  double* g;    // m+1
  double* y;    // m
  double* hcol; // m+2
  double* out;  // 2: |g_{j+1}|, h_{j+1,j}
};

__global__ void k_gmres_init(GmresState s, int m, const double* beta) {
  for (int k = 0; k <= m; ++k) s.g[k] = 0.0;
  s.g[0] = *beta;
}

__global__ void k_givens(GmresState s, int m, int j) {
  double* col = s.H + static_cast<int64_t>(j) * (m + 1);
  for (int i = 0; i <= j + 1; ++i) col[i] = s.hcol[i];
  for (int i = 0; i < j; ++i) {
    double t = s.cs[i] * col[i] + s.sn[i] * col[i + 1];
    col[i + 1] = -s.sn[i] * col[i] + s.cs[i] * col[i + 1];
    col[i] = t;
  }
  double den = hypot(col[j], col[j + 1]);
  double c = den == 0.0 ? 1.0 : col[j] / den;
  double sg = den == 0.0 ? 0.0 : col[j + 1] / den;
  s.cs[j] = c;
  s.sn[j] = sg;
  col[j] = c * col[j] + sg * col[j + 1];
  col[j + 1] = 0.0;
  s.g[j + 1] = -sg * s.g[j];
  s.g[j] = c * s.g[j];
  s.out[0] = fabs(s.g[j + 1]);
  s.out[1] = s.hcol[j + 1];
}

__global__ void k_backsolve(GmresState s, int m, int k) {
  for (int i = k - 1; i >= 0; --i) {
    double t = s.g[i];
    for (int c = i + 1; c < k; ++c) t -= s.H[static_cast<int64_t>(c) * (m + 1) + i] * s.y[c];
    s.y[i] = t / s.H[static_cast<int64_t>(i) * (m + 1) + i];
  }
}

// ---- helpers ------------------------------------------------------------------
struct Work {
  double *r, *w, *d1, *z, *rc, *xc, *part, *V, *Z;
  double* gpart;  // partial sums of the coarse matrix-vector product
  float *r32, *d1_32, *rh32, *x32, *y32;
  double *rh, *x, *y;
  GmresState gs;
  int m;
};

Work work_of(Handle* h) {
  Work k{};
  int64_t n = h->n;
  int m = static_cast<int>((h->wk_vectors - 7) / 2);
  double* b = h->wk.get();
  k.m = m;
  k.r = b;
  k.w = b + n;
  k.d1 = b + 2 * n;
  k.z = b + 3 * n;
  k.rh = b + 4 * n;
  k.x = b + 5 * n;
  k.y = b + 6 * n;
  k.V = b + 7 * n;
  k.Z = k.V + static_cast<int64_t>(m + 1) * n;
  double* s = h->red.get();
  k.part = s;
  k.gpart = h->gpart.get();
  double* hs = h->hred.get();
  k.rc = hs;
  k.xc = hs + h->nc;
  double* q = hs + 2 * h->nc;
  k.gs.H = q;
  q += static_cast<int64_t>(m + 1) * m;
  k.gs.cs = q;
  q += m;
  k.gs.sn = q;
  q += m;
  k.gs.g = q;
  q += m + 1;
  k.gs.y = q;
  q += m;
  k.gs.hcol = q;
  q += m + 2;
  k.gs.out = q;
  if (h->precision == FAMS_PREC_MIXED) {
    float* f = h->wk32.get();
    k.r32 = f;
    k.d1_32 = f + n;
    k.rh32 = f + 2 * n;
    k.x32 = f + 3 * n;
    k.y32 = f + 4 * n;
  }
  return k;
}

// ||a||^2 or a.b into dst (device)
void dot_into(Handle* h, const double* a, const double* b, int64_t n, double* part, double* dst) {
  int nb = std::min<int64_t>(kRedBlocks, blocks_for(n, kT));
  LAUNCH(h, "dot", k_dot_part, nb, kT, 0, n, a, b, part);
  LAUNCH(h, "reduce", k_reduce, 1, 256, 0, nb, 1, 1, part, dst, 0);
}

double read_d(Handle* h, const double* d) {
  double v = 0.0;
  HIPX(hipMemcpyAsync(&v, d, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  return v;
}

double norm_host(Handle* h, const double* a, int64_t n, double* part, double* scratch) {
  dot_into(h, a, a, n, part, scratch);
  return std::sqrt(read_d(h, scratch));
}

template <class TV, class TX, class TB, class TY>
void resid(Handle* h, const TV* val, const TX* x, const TB* b, TY* y) {
  LAUNCH(h, "spmv_resid", (k_resid<TV, TX, TB, TY>), blocks_for(h->n, kT / kSub), kT, 0, h->n,
         h->rp.get(), h->ci.get(), val, x, b, y);
}

// Table 1 steps 5-7 on a residual r (FP64 in, FP64 out); T = stage type
template <class T>
void stage(Handle* h, const Work& k, const double* r, double* z) {
  const int n = h->n, nc = h->nc;
  const T* pv;
  const T* rv;
  const T* av;
  const T* lu;
  const T* rT;
  T *d1, *rh, *x, *ysc;
  if constexpr (std::is_same<T, double>::value) {
    pv = h->p_val.get();
    rv = h->r_val.get();
    av = h->val.get();
    lu = h->ilu.get();
    rT = r;
    d1 = k.d1;
    rh = k.rh;
    x = k.x;
    ysc = k.y;
  } else {
    pv = h->p_val32.get();
    rv = h->r_val32.get();
    av = h->val32.get();
    lu = h->ilu32.get();
    LAUNCH(h, "cast_d2f", (k_cast<double, float>), blocks_for(n, kT), kT, 0, (int64_t)n, r,
           k.r32);
    rT = k.r32;
    d1 = k.d1_32;
    rh = k.rh32;
    x = k.x32;
    ysc = k.y32;
  }
  LAUNCH(h, "restrict", (k_spmv_wave<T, T>), blocks_for(nc, 4), 256, 0, nc, h->r_rp.get(),
         h->r_ci.get(), rv, rT, k.rc);
  coarse_apply(h, h->Ainv.get(), nc, k.rc, k.xc, k.gpart);
  LAUNCH(h, "prolong", (k_spmv8<T, double, T>), blocks_for(n, kT / kSub), kT, 0, n,
         h->p_rp.get(), h->p_ci.get(), pv, k.xc, d1);
  if (h->smoother) {
    resid<T, T, T, T>(h, av, d1, rT, rh);
    ilu_apply<T>(h, lu, rh, x, ysc);
    if (h->blk) {  // per-medium stage: r <- r - A x (row by row, in place), x += M_B^{-1} r
      Handle* b = h->blk.get();
      T* xb;
      const T* blu;
      if constexpr (std::is_same<T, double>::value) {
        xb = h->blk_x.get();
        blu = b->ilu.get();
      } else {
        xb = h->blk_x32.get();
        blu = b->ilu32.get();
      }
      resid<T, T, T, T>(h, av, x, rh, rh);
      ilu_apply<T>(b, blu, rh, xb, ysc);
      LAUNCH(h, "add", (k_add<T, T, T>), blocks_for(n, kT), kT, 0, (int64_t)n, x, xb, x);
    }
    LAUNCH(h, "add", (k_add<T, T, double>), blocks_for(n, kT), kT, 0, (int64_t)n, d1, x, z);
  } else {
    LAUNCH(h, "cast", (k_cast<T, double>), blocks_for(n, kT), kT, 0, (int64_t)n, d1, z);
  }
}

void stage_any(Handle* h, const Work& k, const double* r, double* z) {
  if (h->precision == FAMS_PREC_MIXED) stage<float>(h, k, r, z);
  else stage<double>(h, k, r, z);
}

fams_status_t richardson(Handle* h, const Work& k, const double* q, double* p,
                         const fams_solve_opts_t* o, fams_info_t* info) {
  const int n = h->n;
  double* scratch = k.gs.out;
  resid<double, double, double, double>(h, h->val.get(), p, q, k.r);
  double r0 = norm_host(h, k.r, n, k.part, scratch);
  int it = 0;
  fams_status_t st = FAMS_NOT_CONVERGED;
  double nr = r0;
  if (r0 == 0.0) st = FAMS_OK;
  while (st != FAMS_OK && it < o->max_iter) {
    stage_any(h, k, k.r, k.z);
    LAUNCH(h, "axpy", k_axpy, blocks_for(n, kT), kT, 0, (int64_t)n, 1.0, k.z, p);
    resid<double, double, double, double>(h, h->val.get(), p, q, k.r);
    ++it;
    nr = norm_host(h, k.r, n, k.part, scratch);
    if (!std::isfinite(nr) || nr > 1e8 * r0) {
      st = FAMS_DIVERGED;
      break;
    }
    if (nr <= o->rtol * r0) st = FAMS_OK;
  }
  info->iterations = it;
  info->rel_residual = r0 > 0 ? nr / r0 : 0.0;
  return st;
}

fams_status_t gmres(Handle* h, const Work& k, const double* q, double* p,
                    const fams_solve_opts_t* o, fams_info_t* info) {
  const int64_t n = h->n;
  const int m = std::min(o->restart, k.m);
  double* scratch = k.gs.out;
  resid<double, double, double, double>(h, h->val.get(), p, q, k.r);
  double r0 = norm_host(h, k.r, n, k.part, scratch);
  double tol = o->rtol * r0;
  int it = 0;
  fams_status_t st = FAMS_NOT_CONVERGED;
  const int nb = std::min<int64_t>(kRedBlocks, blocks_for(n, kT));
  double beta = r0;
  while (true) {
    if (beta <= tol) {
      st = FAMS_OK;
      break;
    }
    if (!std::isfinite(beta) || beta > 1e8 * r0) {
      st = FAMS_DIVERGED;
      break;
    }
    if (it >= o->max_iter) break;
    // V_0 = r / beta
    dot_into(h, k.r, k.r, n, k.part, k.gs.hcol + m + 1);
    LAUNCH(h, "sqrt", k_sqrt_into, 1, 1, 0, k.gs.hcol + m + 1, k.gs.hcol + m + 1);
    LAUNCH(h, "scale", k_scale_by, blocks_for(n, kT), kT, 0, n, k.r, k.gs.hcol + m + 1, k.V);
    LAUNCH(h, "gmres_init", k_gmres_init, 1, 1, 0, k.gs, m, k.gs.hcol + m + 1);
    int kk = 0;
    for (int j = 0; j < m; ++j) {
      double* vj = k.V + j * n;
      double* zj = k.Z + j * n;
      stage_any(h, k, vj, zj);
      LAUNCH(h, "spmv", (k_spmv8<double, double, double>), blocks_for(n, kT / kSub), kT, 0,
             (int)n, h->rp.get(), h->ci.get(), h->val.get(), zj, k.w);
      // CGS2 against V_0..V_j: h = V^T w, w -= V h; c = V^T w, w -= V c; h += c
      LAUNCH(h, "mdot", k_mdot_part, nb, kT, 0, n, j + 1, k.V, n, k.w, k.part, m + 2);
      LAUNCH(h, "reduce", k_reduce, j + 1, 256, 0, nb, j + 1, m + 2, k.part, k.gs.hcol, 0);
      LAUNCH(h, "maxpy", k_maxpy, blocks_for(n, kT), kT, 0, n, j + 1, k.V, n, k.gs.hcol, -1.0,
             k.w);
      LAUNCH(h, "mdot", k_mdot_part, nb, kT, 0, n, j + 1, k.V, n, k.w, k.part, m + 2);
      LAUNCH(h, "reduce", k_reduce, j + 1, 256, 0, nb, j + 1, m + 2, k.part, k.gs.y, 0);
      LAUNCH(h, "maxpy", k_maxpy, blocks_for(n, kT), kT, 0, n, j + 1, k.V, n, k.gs.y, -1.0,
             k.w);
      LAUNCH(h, "vadd", k_vadd, 1, 64, 0, j + 1, k.gs.y, k.gs.hcol);
      dot_into(h, k.w, k.w, n, k.part, k.gs.hcol + j + 1);
      LAUNCH(h, "sqrt", k_sqrt_into, 1, 1, 0, k.gs.hcol + j + 1, k.gs.hcol + j + 1);
      LAUNCH(h, "givens", k_givens, 1, 1, 0, k.gs, m, j);
      double est_hn[2];
      HIPX(hipMemcpyAsync(est_hn, k.gs.out, 2 * sizeof(double), hipMemcpyDeviceToHost,
                          h->stream));
      HIPX(hipStreamSynchronize(h->stream));
      ++it;
      kk = j + 1;
      if (est_hn[0] <= tol || it >= o->max_iter || !(est_hn[1] > 0.0) ||
          !std::isfinite(est_hn[0]))
        break;
      LAUNCH(h, "scale", k_scale_by, blocks_for(n, kT), kT, 0, n, k.w, k.gs.hcol + j + 1,
             k.V + (j + 1) * n);
    }
    LAUNCH(h, "backsolve", k_backsolve, 1, 1, 0, k.gs, m, kk);
    LAUNCH(h, "maxpy", k_maxpy, blocks_for(n, kT), kT, 0, n, kk, k.Z, n, k.gs.y, 1.0, p);
    resid<double, double, double, double>(h, h->val.get(), p, q, k.r);
    beta = norm_host(h, k.r, n, k.part, scratch);
  }
  info->iterations = it;
  info->rel_residual = r0 > 0 ? beta / r0 : 0.0;
  return st;
}

// a bounded wait that gave up means the sweep's dependency order was broken
void check_sweeps(Handle* h) {
  if (!h->sweep_err.get()) return;
  int e[2] = {};
  HIPX(hipMemcpyAsync(e, h->sweep_err.get(), sizeof(e), hipMemcpyDeviceToHost, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  h->info.long_waits += e[1];
  HIPX(hipMemsetAsync(h->sweep_err.get() + 1, 0, sizeof(int), h->stream));
  FAMS_REQUIRE(e[0] == 0, FAMS_ERR_DEVICE, "ILU(0) sweep: a dependency wait exceeded its bound");
}

}  // namespace

void ensure_workspace(Handle* h, int restart) {
  int m = std::max(restart, 1);
  size_t need = static_cast<size_t>(7 + 2 * m + 1);
  if (h->wk_vectors >= need) return;
  h->wk.reset(&h->alloc, need * static_cast<size_t>(h->n));
  h->wk_vectors = need;
  h->red.reset(&h->alloc, static_cast<size_t>(kRedBlocks) * (m + 2) + 16);
  h->hred.reset(&h->alloc, 2 * static_cast<size_t>(h->nc) + static_cast<size_t>(m + 1) * m +
                               6 * static_cast<size_t>(m) + 16);
  if (h->precision == FAMS_PREC_MIXED) h->wk32.reset(&h->alloc, 5 * static_cast<size_t>(h->n));
  const size_t nch = (static_cast<size_t>(h->nc) + 63) / 64;   // coarse GEMV column chunks
  if (h->gpart.size() < nch * h->nc) h->gpart.reset(&h->alloc, nch * h->nc);
}

fams_status_t solve_one(Handle* h, const double* q, double* p, const fams_solve_opts_t* o,
                        fams_info_t* info) {
  ensure_workspace(h, o->outer == FAMS_GMRES ? o->restart : 1);
  Work k = work_of(h);
  if (h->sweep_err.get()) HIPX(hipMemsetAsync(h->sweep_err, 0, sizeof(int), h->stream));
  if (!o->use_initial_guess) HIPX(hipMemsetAsync(p, 0, sizeof(double) * h->n, h->stream));
  auto t0 = std::chrono::steady_clock::now();
  fams_status_t st = o->outer == FAMS_GMRES ? gmres(h, k, q, p, o, info)
                                            : richardson(h, k, q, p, o, info);
  HIPX(hipStreamSynchronize(h->stream));
  check_sweeps(h);
  info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                 .count();
  info->status = st;
  return st;
}

void apply_stage_fp64(Handle* h, const double* r, double* z) {
  ensure_workspace(h, 1);
  Work k = work_of(h);
  stage_any(h, k, r, z);
  HIPX(hipStreamSynchronize(h->stream));
  check_sweeps(h);
}

// The stage's scratch inside one caller-provided region of device memory:
// [rc | xc | gpart | d1 rh x y] (FP64 handles) or [rc | xc | gpart | r32 d1
// rh x y] in float (precision form), each part 256-byte aligned.  Returns
// the bytes needed; with `base` != null, also fills `k`.
static size_t stage_scratch_layout(Handle* h, void* base, Work* k) {
  const size_t n = h->n, nc = h->nc, nch = (nc + 63) / 64;
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t o_xc = up(nc * sizeof(double));
  const size_t o_gp = o_xc + up(nc * sizeof(double));
  const size_t o_v = o_gp + up(nch * nc * sizeof(double));
  const bool mixed = h->precision == FAMS_PREC_MIXED;
  const size_t vb = up(n * (mixed ? sizeof(float) : sizeof(double)));
  const size_t total = o_v + (mixed ? 5 : 4) * vb;
  if (base && k) {
    char* b = static_cast<char*>(base);
    *k = Work{};
    k->rc = reinterpret_cast<double*>(b);
    k->xc = reinterpret_cast<double*>(b + o_xc);
    k->gpart = reinterpret_cast<double*>(b + o_gp);
    if (mixed) {
      float* f[5];
      for (int i = 0; i < 5; ++i) f[i] = reinterpret_cast<float*>(b + o_v + i * vb);
      k->r32 = f[0];
      k->d1_32 = f[1];
      k->rh32 = f[2];
      k->x32 = f[3];
      k->y32 = f[4];
    } else {
      double* d[4];
      for (int i = 0; i < 4; ++i) d[i] = reinterpret_cast<double*>(b + o_v + i * vb);
      k->d1 = d[0];
      k->rh = d[1];
      k->x = d[2];
      k->y = d[3];
    }
  }
  return total;
}

size_t stage_scratch_bytes(Handle* h) { return stage_scratch_layout(h, nullptr, nullptr); }

// the stage with its scratch in `base` (stage_scratch_bytes bytes); the
// handle's own structures were all allocated by the setup
void apply_stage_in(Handle* h, void* base, const double* r, double* z) {
  Work k;
  stage_scratch_layout(h, base, &k);
  stage_any(h, k, r, z);
  HIPX(hipStreamSynchronize(h->stream));
  check_sweeps(h);
}

double dev_dot(Handle* h, const double* a, const double* b, int64_t n) {
  ensure_workspace(h, 1);
  Work k = work_of(h);
  dot_into(h, a, b, n, k.part, k.gs.out);
  return read_d(h, k.gs.out);
}

void dev_copy_d(Handle* h, double* dst, const double* src, int64_t n) {
  HIPX(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
}

}  // namespace fams
