// Conservative fine-scale flux reconstruction (Sec. 3.2: a stage with the
// finite-volume restriction R^FV makes a mass-conservative fine-scale flux
// field available; Sec. 4.6).  The paper gives no algorithm; this is the
// standard multiscale finite-volume reconstruction:
//
//  1. FV stage: A_FV = R^FV A P (dense; R^FV sums the cells of a primal
//     block), x = A_FV^{-1} R^FV (q - A p) with two steps of iterative
//     refinement, p' = p + P x: every primal block then conserves mass.
//  2. One Neumann problem per primal block K (one workgroup each, banded
//     LDL^T): fluxes across K's boundary from p', inside from p''
//         sum_{j in K} T_ij (p''_i - p''_j) + s_i p''_i
//             = q_i - sum_{j not in K} T_ij (p'_i - p'_j),     T_ij = -A_ij,
//     s_i = sum_j A_ij.  If no cell of K has s_i > 0 the problem is singular
//     but compatible and p'' is pinned to p' at K's coarse node.
//  3. F_ij = T_ij (p''_i - p''_j) inside a block, T_ij (p'_i - p'_j) across;
//     E_i = s_i p''_i - q_i in the diagonal slot; sum_j F_ij + E_i = 0.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <numeric>
#include <vector>

#include "band.hpp"
#include "order.hpp"
#include "internal.hpp"

namespace fams {
namespace {

constexpr int kT = 256;
// refinement of the FV coarse solve against the fine-scale defect: at least
// kFvRefine steps, then more while the largest primal-block defect still
// halves, at most kFvRefineMax (a block pinned at its coarse node in the
// Neumann problems carries its whole remaining defect at that cell)
constexpr int kFvRefine = 2;
constexpr int kFvRefineMax = 10;
// refinement steps of each block's Neumann solve with its resident factors:
// at a high permeability contrast a block's local matrix is ill conditioned
// and every step gains about -log10(cond * eps) digits of the balance
constexpr int kNeumannRefine = 3;
// a row sum counts as zero (no Dirichlet coupling) when it is rounding:
// |s_i| <= kSingularRowsum * sum_{j != i} |A_ij|, against the row's own
// couplings (a weakly coupled boundary cell beside high-transmissibility
// fractures has a real s_i > 0; pinning its block would leave s_i d_i
// unbalanced at the coarse node)
constexpr double kSingularRowsum = 1e-10;

__global__ void k_rowsum_diag(int n, const int* rp, const int* ci, const double* av, double* s,
                              double* dmax_part) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double dmax = 0.0;
  if (i < n) {
    double t = 0.0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      t += av[p];
      if (ci[p] == i) dmax = av[p];
    }
    s[i] = t;
  }
  __shared__ double red[kT];
  red[threadIdx.x] = dmax;
  __syncthreads();
  for (int k = kT / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + k]);
    __syncthreads();
  }
  if (threadIdx.x == 0) dmax_part[blockIdx.x] = red[0];
}

__global__ void k_max_reduce(int m, const double* part, double* out) {
  __shared__ double red[kT];
  double v = 0.0;
  for (int k = threadIdx.x; k < m; k += blockDim.x) v = fmax(v, part[k]);
  red[threadIdx.x] = v;
  __syncthreads();
  for (int k = kT / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + k]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// *out = max_k |v[k]| (one workgroup)
__global__ void k_absmax(int m, const double* v, double* out) {
  __shared__ double red[kT];
  double a = 0.0;
  for (int k = threadIdx.x; k < m; k += blockDim.x) a = fmax(a, fabs(v[k]));
  red[threadIdx.x] = a;
  __syncthreads();
  for (int k = kT / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + k]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

__global__ void k_iota_f(int n, int* v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = i;
}

__global__ void k_block_ptr(int n, int nb, const int* key_sorted, int* ptr) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  int k = key_sorted[t];
  if (t == 0 || key_sorted[t - 1] != k) ptr[k] = t;
  if (t == n - 1) ptr[nb] = n;
}

__global__ void k_block_local(int n, const int* cells, const int* primal, const int* ptr,
                              int* local) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) local[cells[t]] = t - ptr[primal[cells[t]]];
}

// per primal block: bandwidth of its within-block couplings and whether the
// local Neumann problem is singular (no cell with a positive row sum)
__global__ void k_fv_symbolic(const int* ptr, const int* cells, const int* rp, const int* ci,
                              const double* av, const int* primal, const int* local,
                              const double* s, int* band, int* singular) {
  __shared__ int s_b, s_pos;
  int K = blockIdx.x;
  if (threadIdx.x == 0) {
    s_b = 0;
    s_pos = 0;
  }
  __syncthreads();
  int beg = ptr[K], n = ptr[K + 1] - beg;
  int bm = 0, pos = 0;
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    int i = cells[beg + l];
    double off = 0.0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      int j = ci[p];
      if (j != i) off += fabs(av[p]);
      if (j != i && primal[j] == K) bm = max(bm, abs(local[j] - l));
    }
    if (s[i] > kSingularRowsum * off) pos = 1;
  }
  atomicMax(&s_b, bm);
  atomicOr(&s_pos, pos);
  __syncthreads();
  if (threadIdx.x == 0) {
    band[K] = s_b;
    singular[K] = s_pos ? 0 : 1;
  }
}

__global__ void k_block_sum(int nb, const int* ptr, const int* cells, const double* r,
                            double* out) {
  int K = blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= nb) return;
  double t = 0.0;
  for (int k = ptr[K]; k < ptr[K + 1]; ++k) t += r[cells[k]];
  out[K] = t;
}

__global__ void k_sub(int n, const double* a, const double* b, double* y) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a[i] - b[i];
}

__global__ void k_add_to(int n, const double* a, double* y) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += a[i];
}

// y = b - A x written with the fluxes: b_i - s_i x_i + sum_{j != i} A_ij (x_i -
// x_j) (s = row sums of A); the same value, rounded relative to the fluxes
// rather than to the products A_ij x_j (many orders larger beside
// high-transmissibility fractures)
__global__ void k_resid_f(int n, const int* rp, const int* ci, const double* av, const double* s,
                          const double* x, const double* b, double* y) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xi = x[i];
  double t = b[i] - s[i] * xi;
  for (int p = rp[i]; p < rp[i + 1]; ++p) {
    const int j = ci[p];
    if (j != i) t += av[p] * (xi - x[j]);
  }
  y[i] = t;
}

__global__ void k_prolong_add(int n, const int* prp, const int* pci, const double* pv,
                              const double* x, const double* p, double* y) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double t = 0.0;
  for (int q = prp[i]; q < prp[i + 1]; ++q) t += pv[q] * x[pci[q]];
  y[i] = p[i] + t;
}

// couplings inside primal block K
struct PrimalEdge {
  const int* primal;
  const int* ci;
  __device__ bool operator()(int p, int i, int K) const {
    const int j = ci[p];
    return j != i && primal[j] == K;
  }
};

// Neumann problem of primal block K for the correction d = p'' - p' (p' the
// FV pressure): (A_KK with diagonal A_ii + sum_{j not in K} A_ij) d = q - A p'
// on the block, the right-hand side in flux form
//   q_i - s_i p'_i + sum_{j != i} A_ij (p'_i - p'_j)   (s_i = row sum of A),
// whose terms are of the size of the fluxes (not of A_ij p'_j, which at a
// high permeability contrast are many orders larger), then kNeumannRefine
// steps of iterative refinement with the resident factors.  A block without a
// Dirichlet cell is pinned at its coarse node (d = 0 there).
//
// k_neumann assembles and factors block K (xs: the right-hand side, rs
// second half: a copy of it); the solves, the residual of the first solve
// and the correction p'' = p' + d follow in k_neumann_solve, one wavefront a
// block.  Blocks beyond the wavefront solver's bandwidth are finished in
// k_neumann itself.

// R <- Rq - A_KK X (the modified block matrix; the pinned row is the identity)
__device__ void neumann_residual(int K, int beg, int n, int lv, const int* cells, const int* rp,
                                 const int* ci, const double* av, const int* primal,
                                 const int* local, const double* X, const double* Rq, double* R,
                                 int t0, int dt) {
  for (int l = t0; l < n; l += dt) {
    const int i = cells[beg + l];
    double r = Rq[l];
    if (l == lv) {
      r -= X[l];
    } else {
      double dg = 0.0;
      for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int j = ci[p];
        const double a = av[p];
        if (j == i) {
          dg += a;
        } else if (primal[j] == K) {
          const int lj = local[j];
          if (lj != lv) r -= a * X[lj];
        } else {
          dg += a;
        }
      }
      r -= dg * X[l];
    }
    R[l] = r;
  }
}

__device__ void neumann_update(int beg, int n, const int* cells, const double* p1,
                               const double* X, double* p2, int t0, int dt) {
  for (int l = t0; l < n; l += dt) {
    const int i = cells[beg + l];
    p2[i] = p1[i] + X[l];
  }
}

// X += R (one refinement correction)
__device__ void neumann_accumulate(int n, double* X, const double* R, int t0, int dt) {
  for (int l = t0; l < n; l += dt) X[l] += R[l];
}

__global__ void __launch_bounds__(kT)
k_neumann(const int* ptr, const int* cells, const int* rp, const int* ci, const double* av,
          const int* primal, const int* local, const int* vertex, const int* band,
          const int* singular, const int64_t* band_off, double* band_glob, int lds_elems,
          const double* q, const double* p1, double* xs, double* rs, double* p2, int* err,
          unsigned long long* timing) {
  extern __shared__ double lds[];
  int K = blockIdx.x;
  unsigned long long* tk = timing ? timing + kTickSlots * static_cast<int64_t>(K) : nullptr;
  if (tk && threadIdx.x == 0) tk[0] = wall_clock64();
  int beg = ptr[K], n = ptr[K + 1] - beg;
  int b = band[K], w = b + 1;
  const int64_t bsz = static_cast<int64_t>(n) * w;
  const int mode = band_mode(n, b, lds_elems);
  double* G = band_glob + band_off[K];  // band, then its columns
  double* Lt = G + bsz;
  double* B = mode == 0 ? lds + band_panel_elems(b) : G;
  double* X = xs + beg;
  double* R = rs + beg;                    // residual / correction
  double* Rq = rs + ptr[gridDim.x] + beg;  // the right-hand side, kept
  const bool pin = singular[K] != 0;
  const int lv = pin ? local[vertex[K]] : -1;
  for (int64_t t = threadIdx.x; t < bsz; t += blockDim.x) B[t] = 0.0;
  __syncthreads();
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    const int i = cells[beg + l];
    const double pi = p1[i];
    double dg = 0.0, rs_i = 0.0, rhs = q[i];
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      const int j = ci[p];
      const double a = av[p];
      rs_i += a;
      if (j == i) {
        dg += a;
        continue;
      }
      rhs += a * (pi - p1[j]);
      if (primal[j] == K) {
        const int lj = local[j];
        if (lj < l && lj != lv && l != lv) B[static_cast<int64_t>(l) * w + b - (l - lj)] = a;
      } else {
        dg += a;
      }
    }
    rhs -= rs_i * pi;
    if (l == lv) {
      dg = 1.0;
      rhs = 0.0;
    }
    B[static_cast<int64_t>(l) * w + b] = dg;
    X[l] = rhs;
    Rq[l] = rhs;
  }
  __syncthreads();
  if (tk && threadIdx.x == 0) {
    tk[1] = wall_clock64();
    tk[5] = (static_cast<unsigned long long>(n) << 32) | static_cast<unsigned>(b);
    tk[6] = (1ull << 32) | static_cast<unsigned>(mode);
  }
  bool bad = band_factor<double>(mode, G, Lt, n, b, lds, tk ? tk + 2 : nullptr);
  if (band_wave_class(b) != 0) {
    if (mode == 0) band_export<double>(lds + band_panel_elems(b), G, n, b);
  } else {
    band_substitute<double, double>(B, n, b, X, 1, lds);
    for (int it = 0; it < kNeumannRefine; ++it) {
      __syncthreads();
      neumann_residual(K, beg, n, lv, cells, rp, ci, av, primal, local, X, Rq, R, threadIdx.x,
                       blockDim.x);
      __syncthreads();
      band_substitute<double, double>(B, n, b, R, 1, lds);
      __syncthreads();
      neumann_accumulate(n, X, R, threadIdx.x, blockDim.x);
    }
    __syncthreads();
    neumann_update(beg, n, cells, p1, X, p2, threadIdx.x, blockDim.x);
  }
  if (bad && threadIdx.x == 0) atomicOr(err, 1);
  if (tk && threadIdx.x == 0) tk[4] = wall_clock64();
}

// solves of the Neumann problems of the blocks list[.] (chunk-slot class M)
// with the factors k_neumann left in global memory, one wavefront a block
template <int M>
__global__ void __launch_bounds__(64)
k_neumann_solve(const int* list, int nc, const int* ptr, const int* cells, const int* rp,
                const int* ci, const double* av, const int* primal, const int* local,
                const int* vertex, const int* band, const int* singular,
                const int64_t* band_off, const double* band_glob, const double* p1, double* xs,
                double* rs, double* p2) {
  const int K = list[blockIdx.x];
  const int beg = ptr[K], n = ptr[K + 1] - beg, b = band[K];
  const double* G = band_glob + band_off[K];
  const double* Lt = G + static_cast<int64_t>(n) * (b + 1);
  double* X = xs + beg;
  double* R = rs + beg;
  const double* Rq = rs + ptr[nc] + beg;
  const int lv = singular[K] != 0 ? local[vertex[K]] : -1;
  band_wave_columns<double, double, double, M, 1, 4>(G, Lt, 1, 0, n, b, X, 1, 0, X);
  for (int it = 0; it < kNeumannRefine; ++it) {
    __syncthreads();
    neumann_residual(K, beg, n, lv, cells, rp, ci, av, primal, local, X, Rq, R, threadIdx.x, 64);
    __syncthreads();
    band_wave_columns<double, double, double, M, 1, 4>(G, Lt, 1, 0, n, b, R, 1, 0, R);
    __syncthreads();
    neumann_accumulate(n, X, R, threadIdx.x, 64);
  }
  __syncthreads();
  neumann_update(beg, n, cells, p1, X, p2, threadIdx.x, 64);
}

__global__ void k_flux(int n, const int* rp, const int* ci, const double* av, const int* primal,
                       const double* p1, const double* p2, const double* q, const double* s,
                       double* flux, double* bal_part, double* scale_part) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double bal = 0.0, sc = 0.0;
  if (i < n) {
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      int j = ci[p];
      double f;
      if (j == i) f = s[i] * p2[i] - q[i];
      else if (primal[i] == primal[j]) f = -av[p] * (p2[i] - p2[j]);
      else f = -av[p] * (p1[i] - p1[j]);
      flux[p] = f;
      bal += f;
      sc += fabs(f);
    }
  }
  __shared__ double rb[kT], rs[kT];
  rb[threadIdx.x] = fabs(bal);
  rs[threadIdx.x] = sc;
  __syncthreads();
  for (int k = kT / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) {
      rb[threadIdx.x] = fmax(rb[threadIdx.x], rb[threadIdx.x + k]);
      rs[threadIdx.x] = fmax(rs[threadIdx.x], rs[threadIdx.x + k]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    bal_part[blockIdx.x] = rb[0];
    scale_part[blockIdx.x] = rs[0];
  }
}

}  // namespace

double reconstruct_flux(Handle* h, const double* q, const double* p, double* flux,
                        double* p_fv) {
  const int n = h->n, nc = h->nc;
  Allocator* A = &h->alloc;
  const unsigned g = blocks_for(n, kT);
  ensure_workspace(h, 1);
  // ---- lazy FV setup (kept in the handle) ----
  DBuf<double> s(A, n), dpart(A, g), dmax(A, 2);
  LAUNCH(h, "flux_rowsum", k_rowsum_diag, g, kT, 0, n, h->rp.get(), h->ci.get(), h->val.get(),
         s.get(), dpart.get());
  LAUNCH(h, "flux_max", k_max_reduce, 1, kT, 0, (int)g, dpart.get(), dmax.get());
  DBuf<int> local(A, n), band(A, nc), singular(A, nc);
  if (!h->fv_ready) {
    DBuf<int> keys(A, n), iota(A, n);
    h->fv_order.reset(A, n);
    h->fv_ptr.reset(A, nc + 1);
    LAUNCH(h, "flux_iota", k_iota_f, g, kT, 0, n, iota.get());
    int bits = 1;
    while ((int64_t(1) << bits) <= nc) ++bits;
    sort_pairs_i32(h, h->primal, keys, iota, h->fv_order, n, bits);
    LAUNCH(h, "flux_block_ptr", k_block_ptr, g, kT, 0, n, nc, keys.get(), h->fv_ptr.get());
    {  // breadth-first local order inside each primal block where it narrows
       // the band (fracture blocks whose cells lie on several plates)
      DBuf<int> loc0(A, n);
      LAUNCH(h, "flux_block_local", k_block_local, g, kT, 0, n, h->fv_order.get(),
             h->primal.get(), h->fv_ptr.get(), loc0.get());
      const int cap = order_adj_cap(lds_hw_budget(h));
      allow_lds(reinterpret_cast<const void*>(&k_local_order<PrimalEdge>),
                cap * sizeof(unsigned short));
      LAUNCH(h, "flux_order", k_local_order<PrimalEdge>, nc, kOrderThreads,
             cap * sizeof(unsigned short), h->fv_ptr.get(), h->fv_order.get(), h->rp.get(),
             h->ci.get(), PrimalEdge{h->primal.get(), h->ci.get()}, loc0.get(), cap);
    }
    h->Afv.reset(A, static_cast<size_t>(nc) * nc);
    build_coarse_operator(h, h->fv_ptr, h->fv_order, nullptr, nc, h->Afv);
    // the FV operator is not symmetric: LU with partial pivoting; its three
    // solves per call use the factors (an explicit inverse costs more)
    h->Afv_lu.reset(A, static_cast<size_t>(nc) * nc);
    HIPX(hipMemcpyAsync(h->Afv_lu, h->Afv.get(), sizeof(double) * nc * nc,
                        hipMemcpyDeviceToDevice, h->stream));
    if (nc <= lu_solve_limit()) {
      h->Afv_perm.reset(A, nc);
      lu_factor(h, h->Afv_lu, nc, h->Afv_perm);
    } else {  // too large for the one-workgroup solve: keep the inverse instead
      DBuf<double> inv(A, static_cast<size_t>(nc) * nc);
      lu_inverse(h, h->Afv_lu, inv, nc);
      HIPX(hipMemcpyAsync(h->Afv_lu, inv.get(), sizeof(double) * nc * nc,
                          hipMemcpyDeviceToDevice, h->stream));
      HIPX(hipStreamSynchronize(h->stream));
    }
    h->fv_ready = true;
  }
  LAUNCH(h, "flux_block_local", k_block_local, g, kT, 0, n, h->fv_order.get(), h->primal.get(),
         h->fv_ptr.get(), local.get());
  LAUNCH(h, "flux_symbolic", k_fv_symbolic, nc, kT, 0, h->fv_ptr.get(), h->fv_order.get(),
         h->rp.get(), h->ci.get(), h->val.get(), h->primal.get(), local.get(), s.get(),
         band.get(), singular.get());
  std::vector<int> hb(nc), hp(nc + 1);
  HIPX(hipMemcpyAsync(hb.data(), band.get(), nc * sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPX(hipMemcpyAsync(hp.data(), h->fv_ptr.get(), (nc + 1) * sizeof(int), hipMemcpyDeviceToHost,
                      h->stream));
  HIPX(hipStreamSynchronize(h->stream));

  // ---- FV stage ----
  DBuf<double> r(A, n), rc(A, nc), x(A, nc), t(A, nc), t2(A, nc), p1(A, n), p2(A, n), xs(A, n),
      rs(A, 2 * static_cast<size_t>(n));
  LAUNCH(h, "flux_resid", k_resid_f, g, kT, 0, n, h->rp.get(), h->ci.get(), h->val.get(), s.get(),
         p, q, r.get());
  LAUNCH(h, "flux_restrict", k_block_sum, blocks_for(nc, kT), kT, 0, nc, h->fv_ptr.get(),
         h->fv_order.get(), r.get(), rc.get());
  auto fv_solve = [&](const double* in, double* out) {
    if (h->Afv_perm.get()) lu_solve(h, h->Afv_lu, h->Afv_perm, nc, in, out);
    else coarse_apply(h, h->Afv_lu, nc, in, out, h->gpart);   // holds the inverse
  };
  fv_solve(rc, x);
  // iterative refinement against the fine-scale defect R^FV (q - A p'), with
  // p' = p + P x: it removes the coarse solve's error and the rounding of the
  // dense FV operator itself, which bounds the blocks' conservation
  double prev = 0.0;
  for (int it = 0; it < kFvRefineMax; ++it) {
    LAUNCH(h, "flux_prolong", k_prolong_add, g, kT, 0, n, h->p_rp.get(), h->p_ci.get(),
           h->p_val.get(), x.get(), p, p1.get());
    LAUNCH(h, "flux_resid", k_resid_f, g, kT, 0, n, h->rp.get(), h->ci.get(), h->val.get(),
           s.get(), p1.get(), q, r.get());
    LAUNCH(h, "flux_restrict", k_block_sum, blocks_for(nc, kT), kT, 0, nc, h->fv_ptr.get(),
           h->fv_order.get(), r.get(), t.get());
    if (it >= kFvRefine) {  // keep refining only while the block defects still halve
      double m = 0.0;
      LAUNCH(h, "flux_max", k_absmax, 1, kT, 0, nc, t.get(), dmax.get() + 1);
      HIPX(hipMemcpyAsync(&m, dmax.get() + 1, sizeof(double), hipMemcpyDeviceToHost, h->stream));
      HIPX(hipStreamSynchronize(h->stream));
      if (!(m < 0.5 * prev)) break;
      prev = m;
    } else if (it == kFvRefine - 1) {
      LAUNCH(h, "flux_max", k_absmax, 1, kT, 0, nc, t.get(), dmax.get() + 1);
      HIPX(hipMemcpyAsync(&prev, dmax.get() + 1, sizeof(double), hipMemcpyDeviceToHost,
                          h->stream));
    }
    fv_solve(t, t2);
    LAUNCH(h, "flux_add", k_add_to, blocks_for(nc, kT), kT, 0, nc, t2.get(), x.get());
  }
  LAUNCH(h, "flux_prolong", k_prolong_add, g, kT, 0, n, h->p_rp.get(), h->p_ci.get(),
         h->p_val.get(), x.get(), p, p1.get());

  // ---- Neumann problems per primal block ----
  std::vector<int64_t> off(nc, 0);
  int64_t total = 0, lds_need = 0;
  const int64_t lds_cap = lds_budget(h) / static_cast<int64_t>(sizeof(double));
  for (int K = 0; K < nc; ++K) {
    const int nk = hp[K + 1] - hp[K];
    const int mode = band_mode(nk, hb[K], lds_cap);
    FAMS_REQUIRE(mode >= 0, FAMS_ERR_CAPACITY, "primal block bandwidth too large for LDS");
    off[K] = total;
    total += 2 * static_cast<int64_t>(nk) * (hb[K] + 1);  // factor band and Lt
    lds_need = std::max(lds_need, band_lds_elems(mode, nk, hb[K]));
  }
  DBuf<int64_t> d_off(A, nc);
  HIPX(hipMemcpyAsync(d_off, off.data(), nc * sizeof(int64_t), hipMemcpyHostToDevice, h->stream));
  DBuf<double> scratch(A, std::max<int64_t>(total, 1));
  DBuf<int> err(A, 1);
  HIPX(hipMemsetAsync(err, 0, sizeof(int), h->stream));
  allow_lds(reinterpret_cast<const void*>(&k_neumann), lds_need * sizeof(double));
  static const bool timing_on = std::getenv("FAMS_BLOCK_TIMING") != nullptr;
  DBuf<unsigned long long> timing;
  if (timing_on) {
    timing.reset(A, kTickSlots * static_cast<size_t>(nc));
    HIPX(hipMemsetAsync(timing, 0, kTickSlots * nc * sizeof(unsigned long long), h->stream));
  }
  LAUNCH(h, "flux_neumann", k_neumann, nc, kT, lds_need * sizeof(double), h->fv_ptr.get(),
         h->fv_order.get(), h->rp.get(), h->ci.get(), h->val.get(), h->primal.get(), local.get(),
         h->vertex.get(), band.get(), singular.get(), d_off.get(), scratch.get(),
         static_cast<int>(lds_need), q, p1.get(), xs.get(), rs.get(), p2.get(), err.get(),
         timing.get());
  if (timing_on) {
    HIPX(hipStreamSynchronize(h->stream));
    print_block_timing(timing.get(), nc, 0);
  }
  {  // the solves, by chunk-slot class
    std::vector<int> list;
    std::vector<std::pair<int, int>> cls;
    std::vector<int> order(nc);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return hp[a + 1] - hp[a] > hp[b + 1] - hp[b]; });
    for (int m : {2, 3, 4, 5, 6, 7, 9}) {
      const size_t l0 = list.size();
      for (int K : order)
        if (band_wave_class(hb[K]) == m) list.push_back(K);
      if (list.size() > l0) cls.emplace_back(m, static_cast<int>(list.size() - l0));
    }
    DBuf<int> d_list(A, std::max<size_t>(list.size(), 1));
    if (!list.empty())
      HIPX(hipMemcpyAsync(d_list, list.data(), list.size() * sizeof(int), hipMemcpyHostToDevice,
                          h->stream));
    int l0 = 0;
    Fork fork(h);
    for (auto [m, cnt] : cls) {
      hipStream_t st = fork.next();
#define FAMS_NSOLVE(M)                                                                        \
  LAUNCH_ON(h, st, "flux_neumann_solve", k_neumann_solve<M>, cnt, 64, 0,                      \
         static_cast<const int*>(d_list.get() + l0), nc, h->fv_ptr.get(), h->fv_order.get(),   \
         h->rp.get(), h->ci.get(), h->val.get(), h->primal.get(), local.get(), h->vertex.get(), \
         band.get(), singular.get(), d_off.get(), static_cast<const double*>(scratch.get()),    \
         p1.get(), xs.get(), rs.get(), p2.get())
      switch (m) {
        case 2: FAMS_NSOLVE(2); break;
        case 3: FAMS_NSOLVE(3); break;
        case 4: FAMS_NSOLVE(4); break;
        case 5: FAMS_NSOLVE(5); break;
        case 6: FAMS_NSOLVE(6); break;
        case 7: FAMS_NSOLVE(7); break;
        default: FAMS_NSOLVE(9); break;
      }
#undef FAMS_NSOLVE
      l0 += cnt;
    }
    fork.join();
    HIPX(hipStreamSynchronize(h->stream));  // d_list is freed on return
  }

  // ---- fluxes and balance ----
  DBuf<double> bpart(A, g), spart(A, g), mx(A, 2);
  LAUNCH(h, "flux_eval", k_flux, g, kT, 0, n, h->rp.get(), h->ci.get(), h->val.get(),
         h->primal.get(), p1.get(), p2.get(), q, s.get(), flux, bpart.get(), spart.get());
  LAUNCH(h, "flux_max", k_max_reduce, 1, kT, 0, (int)g, bpart.get(), mx.get());
  LAUNCH(h, "flux_max", k_max_reduce, 1, kT, 0, (int)g, spart.get(), mx.get() + 1);
  if (p_fv)
    HIPX(hipMemcpyAsync(p_fv, p1.get(), n * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  double hm[2];
  int he = 0;
  HIPX(hipMemcpyAsync(hm, mx.get(), 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPX(hipMemcpyAsync(&he, err.get(), sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  FAMS_REQUIRE(he == 0, FAMS_ERR_SINGULAR_LOCAL, "non-positive pivot in a block Neumann problem");
  return hm[1] > 0 ? hm[0] / hm[1] : 0.0;
}

}  // namespace fams
