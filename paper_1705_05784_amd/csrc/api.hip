// The C ABI of include/fams.h: argument checks, ownership, error mapping and
// the setup orchestration.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <initializer_list>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

namespace fams {

static thread_local std::string g_last_error;

[[noreturn]] void hip_fail(hipError_t e, const char* what, const char* file, int line) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e) + " (" + file + ":" +
                  std::to_string(line) + ")";
  throw Error(e == hipErrorOutOfMemory ? FAMS_ERR_OOM : FAMS_ERR_DEVICE, m);
}

void* Allocator::alloc(size_t bytes) {
  void* p = nullptr;
  if (has_hook) {
    p = hook.alloc(hook.ctx, bytes, stream);
    if (!p) throw Error(FAMS_ERR_OOM, "allocator hook returned NULL");
  } else {
    hipError_t e = hipMallocAsync(&p, bytes, stream);
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      throw Error(FAMS_ERR_OOM, "hipMallocAsync of " + std::to_string(bytes) + " bytes failed");
    }
  }
  live_bytes += static_cast<int64_t>(bytes);
  peak_bytes = std::max(peak_bytes, live_bytes);
  return p;
}

void Allocator::release(void* p, size_t bytes) {
  if (!p) return;
  if (has_hook) hook.free(hook.ctx, p, stream);
  else (void)hipFreeAsync(p, stream);
  live_bytes -= static_cast<int64_t>(bytes);
}

int Prof::begin(const char* name, hipStream_t s) {
  if (!on) return -1;
  Pending pe;
  pe.name = name;
  pe.s = s ? s : stream;
  HIPX(hipEventCreate(&pe.a));
  HIPX(hipEventCreate(&pe.b));
  HIPX(hipEventRecord(pe.a, pe.s));
  pending.push_back(pe);
  return static_cast<int>(pending.size()) - 1;
}

void Prof::end(int token) {
  if (token < 0) return;
  HIPX(hipEventRecord(pending[token].b, pending[token].s));
  if (pending.size() > 20000 && pending[token].s == stream) collect();
}

void Prof::collect() {
  if (pending.empty()) return;
  HIPX(hipStreamSynchronize(stream));
  for (auto& pe : pending) {
    float ms = 0.f;
    HIPX(hipEventElapsedTime(&ms, pe.a, pe.b));
    auto& t = totals[pe.name];
    t.first += ms;
    t.second += 1;
    (void)hipEventDestroy(pe.a);
    (void)hipEventDestroy(pe.b);
  }
  pending.clear();
}

Prof::~Prof() {
  for (auto& pe : pending) {
    (void)hipEventDestroy(pe.a);
    (void)hipEventDestroy(pe.b);
  }
}

AuxStreams::~AuxStreams() {
  for (int i = 0; i < kAuxStreams; ++i) {
    if (s[i]) {
      (void)hipStreamSynchronize(s[i]);
      (void)hipStreamDestroy(s[i]);
    }
    if (join[i]) (void)hipEventDestroy(join[i]);
  }
  if (fork) (void)hipEventDestroy(fork);
  for (hipEvent_t e : step)
    if (e) (void)hipEventDestroy(e);
}

Fork::Fork(Handle* h) : h_(h) {
  AuxStreams& a = h->aux;
  if (!a.fork) {
    HIPX(hipEventCreateWithFlags(&a.fork, hipEventDisableTiming));
    for (int i = 0; i < kAuxStreams; ++i) {
      HIPX(hipStreamCreateWithFlags(&a.s[i], hipStreamNonBlocking));
      HIPX(hipEventCreateWithFlags(&a.join[i], hipEventDisableTiming));
    }
    for (hipEvent_t& e : a.step) HIPX(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  HIPX(hipEventRecord(a.fork, h->stream));
}

hipStream_t Fork::next() {
  const int i = k_++ % (kAuxStreams + 1);
  if (i == 0) return h_->stream;
  if (!used_[i - 1]) {
    HIPX(hipStreamWaitEvent(h_->aux.s[i - 1], h_->aux.fork, 0));
    used_[i - 1] = true;
  }
  return h_->aux.s[i - 1];
}

void Fork::join() {
  if (joined_) return;
  joined_ = true;
  for (int i = 0; i < kAuxStreams; ++i) {
    if (!used_[i]) continue;
    HIPX(hipEventRecord(h_->aux.join[i], h_->aux.s[i]));
    HIPX(hipStreamWaitEvent(h_->stream, h_->aux.join[i], 0));
  }
}

Fork::~Fork() {
  if (joined_) return;
  joined_ = true;
  for (int i = 0; i < kAuxStreams; ++i) {
    if (!used_[i]) continue;
    (void)hipEventRecord(h_->aux.join[i], h_->aux.s[i]);
    (void)hipStreamWaitEvent(h_->stream, h_->aux.join[i], 0);
  }
}

static double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

PhaseTimer::PhaseTimer(hipStream_t s)
    : stream(s), on(std::getenv("FAMS_SETUP_TIMING") != nullptr), t_last(now_ms()) {}

void PhaseTimer::mark(const char* what) {
  if (!on) return;
  HIPX(hipStreamSynchronize(stream));
  const double t = now_ms();
  std::fprintf(stderr, "[setup] %-22s %8.2f ms\n", what, t - t_last);
  t_last = t;
}

int64_t lds_budget(Handle* h) {
  if (!h->lds_bytes) {
    int dev = 0, v = 0;
    HIPX(hipGetDevice(&dev));
    HIPX(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    // leave room for the kernels' static LDS
    h->lds_bytes = std::min<int64_t>(std::max(v, 65536), 160 * 1024) - 4096;
    h->lds_hw_bytes = h->lds_bytes;
    // FAMS_LDS_LIMIT (bytes) lowers the budget, which moves local blocks to
    // the global-memory storage modes (used to exercise those modes on small
    // problems)
    if (const char* e = std::getenv("FAMS_LDS_LIMIT")) {
      const long long lim = std::atoll(e);
      if (lim > 0) h->lds_bytes = std::min<int64_t>(h->lds_bytes, lim);
    }
  }
  return h->lds_bytes;
}

int64_t lds_hw_budget(Handle* h) {
  lds_budget(h);
  return h->lds_hw_bytes;
}

// The dynamic-LDS limit is process-wide state of the kernel: it is only ever
// raised, under a lock, so that one handle's setting can never lower the
// limit under another thread's launch of the same kernel.
void allow_lds(const void* kernel, size_t bytes) {
  if (bytes <= 65536) return;
  static std::mutex mu;
  static std::unordered_map<const void*, size_t> limit;
  std::lock_guard<std::mutex> lock(mu);
  size_t& cur = limit[kernel];
  if (bytes <= cur) return;
  HIPX(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                           static_cast<int>(bytes)));
  cur = bytes;
}

namespace {

__global__ void k_rowptr_i32(int64_t n, const int64_t* src, int* dst, int* err) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i > n) return;
  int64_t v = src[i];
  if (v < 0 || v > INT32_MAX) atomicOr(err, 1);
  dst[i] = static_cast<int>(v);
  if (i < n && src[i + 1] < v) atomicOr(err, 2);
}

__global__ void k_vertex_i32(int64_t n, const int64_t* src, int* dst) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = static_cast<int>(src[i]);
}

__global__ void k_cols_check(int64_t nnz, int n, const int* ci, int* err) {
  int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < nnz && (ci[p] < 0 || ci[p] >= n)) atomicOr(err, 4);
}

__global__ void k_d2f_api(int64_t n, const double* a, float* b) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) b[i] = static_cast<float>(a[i]);
}

}  // namespace

// an array the kernels read or write must be memory the device can address
// (device, managed or pinned host memory); pageable host memory is refused
// before any work is issued
bool device_addressable(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a{};
  const hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    g_last_error = std::string("an array argument is not memory the device can address "
                               "(hipPointerGetAttributes: ") + hipGetErrorString(e) + ")";
    return false;
  }
  if (a.devicePointer != nullptr || a.isManaged != 0) return true;
  g_last_error = "an array argument is host memory the device cannot address";
  return false;
}

bool all_addressable(std::initializer_list<const void*> ps) {
  for (const void* p : ps)
    if (!device_addressable(p)) return false;
  return true;
}

namespace {

fams_status_t fail(const Error& e) {
  g_last_error = e.what();
  return e.status;
}

template <class F>
fams_status_t guard(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    return fail(e);
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return FAMS_ERR_OOM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return FAMS_ERR_DEVICE;
  }
}

}  // namespace

fams_status_t guarded(const std::function<fams_status_t()>& f) { return guard(f); }

namespace {

// A_c = R A P and its inverse, and the FP32 copy of A (precision form): the
// parts of the setup that follow the values of A for a fixed basis
void coarse_setup(Handle* h) {
  Allocator* al = &h->alloc;
  h->ap_state = 0;  // A P follows A and P
  const int nc = h->nc;
  h->Ac.reset(al, static_cast<size_t>(nc) * nc);
  build_coarse_operator(h, h->r_rp, h->r_ci, h->r_val, nc, h->Ac);
  {
    // A_c = P^T A P is SPD for SPD A: Gauss-Jordan without pivoting; if a
    // pivot is not positive, the restriction is not P^T or A is not
    // symmetric, LU with partial pivoting
    h->Ainv.reset(al, static_cast<size_t>(nc) * nc);
    if (h->restriction != FAMS_RESTRICT_FE || h->nonsym || !spd_inverse(h, h->Ac, h->Ainv, nc)) {
      DBuf<double> lu(al, static_cast<size_t>(nc) * nc);
      HIPX(hipMemcpyAsync(lu, h->Ac.get(), sizeof(double) * nc * nc, hipMemcpyDeviceToDevice,
                          h->stream));
      lu_inverse(h, lu, h->Ainv, nc);
    }
    HIPX(hipStreamSynchronize(h->stream));
  }
  h->ell.val.free();    // the lock-step products' copies of A's values
  h->ell.val32.free();
  if (h->precision == FAMS_PREC_MIXED) {
    h->val32.reset(al, h->nnz);
    LAUNCH(h, "d2f", k_d2f_api, blocks_for(h->nnz, 256), 256, 0, h->nnz, h->val.get(),
           h->val32.get());
  }
  HIPX(hipStreamSynchronize(h->stream));
}

// largest relative change |a_new - a_old| / |a_old| over the entries of A
// (absolute where a_old = 0), as the bits of a non-negative double, so that
// an integer maximum orders them (NaN sorts above every number)
__global__ void k_rel_change(int64_t nnz, const double* a_new, const double* a_old,
                             unsigned long long* out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  const double d = fabs(a_new[i] - a_old[i]);
  const double r = a_old[i] != 0.0 ? d / fabs(a_old[i]) : d;
  atomicMax(out, static_cast<unsigned long long>(__double_as_longlong(r)));
}

// New values of A on the setup's pattern (Table 1, steps 2 and 4; Sec. 3.1:
// the basis functions are updated only when the fine-scale properties
// change beyond a threshold).  The ILU(0) factors, A_c and its inverse
// always follow the new A; P (and R) are recomputed when the largest
// relative change since the last basis exceeds `threshold`.
void update_impl(Handle* h, const double* val, double threshold, int* recomputed) {
  Allocator* al = &h->alloc;
  HIPX(hipMemcpyAsync(h->val, val, h->nnz * sizeof(double), hipMemcpyDeviceToDevice,
                      h->stream));
  DBuf<unsigned long long> mx(al, 1);
  HIPX(hipMemsetAsync(mx, 0, sizeof(unsigned long long), h->stream));
  LAUNCH(h, "update", k_rel_change, blocks_for(h->nnz, 256), 256, 0, h->nnz, h->val.get(),
         h->val_basis.get(), mx.get());
  unsigned long long bits = 0;
  HIPX(hipMemcpyAsync(&bits, mx.get(), sizeof(bits), hipMemcpyDeviceToHost, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  double change;
  std::memcpy(&change, &bits, sizeof(change));
  const bool basis = !(change <= threshold);
  build_ilu(h);
  if (h->smoother == 2) build_block_smoother(h);
  if (basis) {
    build_prolongation(h, h->wb.get());
    if (h->restriction != FAMS_RESTRICT_FE) build_restriction(h);
    HIPX(hipMemcpyAsync(h->val_basis, h->val.get(), h->nnz * sizeof(double),
                        hipMemcpyDeviceToDevice, h->stream));
  }
  coarse_setup(h);
  h->fv_ready = false;  // the FV operator of the flux stage follows A: rebuilt on next use
  HIPX(hipStreamSynchronize(h->stream));
  *recomputed = basis ? 1 : 0;
}

void setup_impl(Handle* h, const fams_csr_t* A, const fams_grid_t* G) {
  auto t0 = std::chrono::steady_clock::now();
  const int64_t n = A->n;
  Allocator* al = &h->alloc;
  DBuf<int> err(al, 1);
  HIPX(hipMemsetAsync(err, 0, sizeof(int), h->stream));
  h->rp.reset(al, n + 1);
  h->ci.reset(al, A->nnz);
  h->val.reset(al, A->nnz);
  LAUNCH(h, "copy_in", k_rowptr_i32, blocks_for(n + 1, 256), 256, 0, n, A->row_ptr, h->rp.get(),
         err.get());
  HIPX(hipMemcpyAsync(h->ci, A->col_idx, A->nnz * sizeof(int), hipMemcpyDeviceToDevice,
                      h->stream));
  HIPX(hipMemcpyAsync(h->val, A->val, A->nnz * sizeof(double), hipMemcpyDeviceToDevice,
                      h->stream));
  LAUNCH(h, "copy_in", k_cols_check, blocks_for(A->nnz, 256), 256, 0, A->nnz, (int)n, h->ci.get(),
         err.get());
  h->wb.reset(al, n);
  HIPX(hipMemcpyAsync(h->wb, G->wb_type, n, hipMemcpyDeviceToDevice, h->stream));
  const int8_t* wb = h->wb.get();
  h->primal.reset(al, n);
  HIPX(hipMemcpyAsync(h->primal, G->primal, n * sizeof(int), hipMemcpyDeviceToDevice, h->stream));
  h->vertex.reset(al, h->nc);
  LAUNCH(h, "copy_in", k_vertex_i32, blocks_for(h->nc, 256), 256, 0, (int64_t)h->nc, G->vertex,
         h->vertex.get());
  int e = 0;
  int64_t last = 0;
  HIPX(hipMemcpyAsync(&e, err.get(), sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPX(hipMemcpyAsync(&last, A->row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  FAMS_REQUIRE(e == 0 && last == A->nnz, FAMS_ERR_INVALID_ARG, "malformed CSR");

  PhaseTimer pt(h->stream);
  pt.mark("validate");
  build_ilu(h);                 // diagonal positions (+ ILU(0) factors)
  if (h->smoother == 2) build_block_smoother(h);  // ILU(0) of diag(A^mm, A^ff)
  pt.mark("ilu");
  build_prolongation(h, wb);    // P, R = P^T
  if (h->restriction != FAMS_RESTRICT_FE) build_restriction(h);  // MSFV / MSMIX rows of R
  pt.mark("prolongation");
  coarse_setup(h);
  pt.mark("coarse inverse");
  h->val_basis.reset(al, h->nnz);
  HIPX(hipMemcpyAsync(h->val_basis, h->val.get(), h->nnz * sizeof(double),
                      hipMemcpyDeviceToDevice, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  const int nc = h->nc;
  h->info.n = n;
  h->info.n_matrix = h->nm;
  h->info.nnz = h->nnz;
  h->info.n_coarse = nc;
  h->info.ms_setup =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace
}  // namespace fams

using fams::Error;
using fams::Handle;

extern "C" {

const char* fams_status_string(fams_status_t s) {
  switch (s) {
    case FAMS_OK: return "ok";
    case FAMS_NOT_CONVERGED: return "not converged (max_iter reached)";
    case FAMS_DIVERGED: return "diverged";
    case FAMS_ERR_INVALID_ARG: return "invalid argument";
    case FAMS_ERR_BAD_GRID: return "inconsistent coarse grid";
    case FAMS_ERR_SINGULAR_LOCAL: return "singular local (basis) problem";
    case FAMS_ERR_SINGULAR_COARSE: return "singular coarse system";
    case FAMS_ERR_ZERO_PIVOT_ILU: return "non-positive ILU(0) pivot";
    case FAMS_ERR_OOM: return "out of device memory";
    case FAMS_ERR_DEVICE: return "HIP runtime error";
    case FAMS_ERR_CAPACITY: return "internal per-block capacity exceeded";
  }
  return "unknown status";
}

/* Last error message of the calling thread (diagnostics; not in fams.h). */
const char* fams_last_error(void) { return fams::g_last_error.c_str(); }

fams_status_t fams_footprint(int64_t n, int64_t nnz, int64_t n_coarse, int32_t precision,
                             int32_t restart, int32_t max_nrhs, size_t* bytes) {
  if (!bytes || n <= 0 || nnz <= 0 || n_coarse <= 0 || max_nrhs < 1 || restart < 1)
    return FAMS_ERR_INVALID_ARG;
  const double zp = 16.0 * n;  // nnz(P) bound used for admission (<= 16 per row)
  const double nc = static_cast<double>(n_coarse);
  const bool mixed = precision == FAMS_PREC_MIXED;
  double b = 0;
  b += nnz * (4 + 8 + 8) + (n + 1) * 4 + n * (4 + 4 + 4);       // A, ILU, diag, primal
  b += nnz * 8.0 + n;                                            // basis values, classes
  b += 2 * zp * (4 + 8) + (n + 2 * nc + 2) * 4;                  // P and R
  b += 2.0 * 8 * nc * nc;                                        // A_c and its inverse
  b += 2.0 * 8 * 1024 * nc + 8.0 * 1024 * 1024;                   // block Gauss-Jordan panels
  b += 3.0 * zp * (4 + 8) + 8.0 * (n + 1);                       // A P
  b += 48.0 * 8 * n;                                             // local solutions (setup)
  b += 2.0 * (4 + 32 + 32 + 4 + 4 + 72 + 8) * n + 24.0 * n;     // sweep schedules, levels
  b += 240.0 * n;                                                // factorisation records
  b += nnz * 24.0 + n * 400.0;                                   // per-medium stage (smoother 2)
  b += 8.0 * n * (6 + 2 * restart + 1);                          // iteration vectors
  if (mixed) b += nnz * 8.0 + 2 * zp * 4 + 16.0 * n;
  if (max_nrhs > 1) {  // lock-step groups of K right-hand sides
    int K = 2;
    while (K < 32 && K < max_nrhs) K *= 2;
    const double nk = static_cast<double>(n) * K;
    b += nk * 8 * (10 + 2 * restart + 1) + (mixed ? nk * 4 * 6 : 0.0);
    b += (2 + 34) * nc * K * 8 + 2048.0 * (2 * restart + 4) * K * 8;
    b += 2 * (n * (8 * (4 + 8) + 8.0) + (mixed ? n * 8 * 4.0 : 0.0));  // A, P in fixed width
  }
  b *= 1.10;
  *bytes = static_cast<size_t>(b) + (64u << 20);
  return FAMS_OK;
}

fams_status_t fams_setup(const fams_csr_t* A, const fams_grid_t* G, const fams_setup_opts_t* o,
                         const fams_allocator_t* allocator, void* stream, fams_handle_t* out) {
  if (out) *out = nullptr;
  if (!A || !G || !o || !out || !A->row_ptr || !A->col_idx || !A->val || !G->wb_type ||
      !G->primal || !G->vertex)
    return FAMS_ERR_INVALID_ARG;
  if (A->n <= 0 || A->n >= (int64_t(1) << 31) || A->nnz < A->n || A->nnz >= (int64_t(1) << 31) ||
      A->n_matrix < 0 || A->n_matrix > A->n || A->n_wells < 0 ||
      A->n_wells > A->n - A->n_matrix || G->n_coarse <= 0 || G->n_coarse > A->n ||
      G->n_coarse > 65536)
    return FAMS_ERR_INVALID_ARG;
  if (o->variant < 0 || o->variant > 3 || o->precision < 0 || o->precision > 1 ||
      !(o->trunc_alpha >= 0.0 && o->trunc_alpha < 1.0) || o->merge_cap < 1 ||
      o->restriction < FAMS_RESTRICT_FE || o->restriction > FAMS_RESTRICT_MIX ||
      o->smoother < 0 || o->smoother > 2 || o->nonsymmetric < 0 || o->nonsymmetric > 1)
    return FAMS_ERR_INVALID_ARG;
  if (!fams::all_addressable({A->row_ptr, A->col_idx, A->val, G->wb_type, G->primal, G->vertex}))
    return FAMS_ERR_INVALID_ARG;
  return fams::guard([&]() -> fams_status_t {
    std::unique_ptr<fams_handle_s> h(new fams_handle_s());
    h->stream = static_cast<hipStream_t>(stream);
    h->alloc.stream = h->stream;
    h->prof.stream = h->stream;
    if (allocator && allocator->alloc && allocator->free) {
      h->alloc.hook = *allocator;
      h->alloc.has_hook = true;
    }
    h->variant = o->variant;
    h->precision = o->precision;
    h->alpha = o->trunc_alpha;
    h->merge_cap = o->merge_cap;
    h->smoother = o->smoother;
    h->restriction = o->restriction;
    h->nonsym = o->nonsymmetric != 0;
    h->prof.on = o->profile != 0;
    h->n = static_cast<int>(A->n);
    h->nm = static_cast<int>(A->n_matrix);
    h->nw = static_cast<int>(A->n_wells);
    h->nnz = A->nnz;
    h->nc = static_cast<int>(G->n_coarse);
    fams::setup_impl(h.get(), A, G);
    h->info.device_bytes = h->alloc.live_bytes + (h->blk ? h->blk->alloc.live_bytes : 0);
    h->info.peak_device_bytes = h->alloc.peak_bytes + (h->blk ? h->blk->alloc.peak_bytes : 0);
    *out = h.release();
    return FAMS_OK;
  });
}

fams_status_t fams_update_values(fams_handle_t h, const double* val, double threshold,
                                 int32_t* basis_recomputed) {
  if (!h || !val || !basis_recomputed || !fams::device_addressable(val))
    return FAMS_ERR_INVALID_ARG;
  return fams::guard([&]() -> fams_status_t {
    int rec = 0;
    fams::update_impl(h, val, threshold, &rec);
    *basis_recomputed = rec;
    h->info.device_bytes = h->alloc.live_bytes + (h->blk ? h->blk->alloc.live_bytes : 0);
    return FAMS_OK;
  });
}

fams_status_t fams_solve(fams_handle_t h, const double* q, double* p, int32_t nrhs,
                         const fams_solve_opts_t* o, fams_info_t* info) {
  if (!h || !q || !p || nrhs < 0 || !o) return FAMS_ERR_INVALID_ARG;
  if (o->outer != FAMS_RICHARDSON && o->outer != FAMS_GMRES) return FAMS_ERR_INVALID_ARG;
  if (o->outer == FAMS_GMRES && (o->restart < 1 || o->restart > 60)) return FAMS_ERR_INVALID_ARG;
  if (!(o->rtol >= 0.0) || o->max_iter < 0) return FAMS_ERR_INVALID_ARG;
  if (nrhs > 0 && !fams::all_addressable({q, p})) return FAMS_ERR_INVALID_ARG;
  return fams::guard([&]() -> fams_status_t {
    fams_status_t worst = FAMS_OK;
    const int64_t n = h->n;
    if (nrhs > 1) {  // several right-hand sides: lock-step groups on the one setup
      std::vector<fams_info_t> inf(nrhs);
      for (int r = 0; r < nrhs; ++r) {
        const double qq = fams::dev_dot(h, q + r * n, q + r * n, n);
        if (!std::isfinite(qq)) {
          inf[r].status = FAMS_ERR_INVALID_ARG;
          if (info) info[r] = inf[r];
          return FAMS_ERR_INVALID_ARG;
        }
      }
      worst = fams::solve_block(h, q, p, nrhs, o, inf.data());
      if (info)
        for (int r = 0; r < nrhs; ++r) info[r] = inf[r];
      return worst;
    }
    for (int r = 0; r < nrhs; ++r) {
      const double* qr = q + r * n;
      double* pr = p + r * n;
      fams_info_t inf{};
      double qq = fams::dev_dot(h, qr, qr, n);
      if (!std::isfinite(qq)) {
        inf.status = FAMS_ERR_INVALID_ARG;
        if (info) info[r] = inf;
        return FAMS_ERR_INVALID_ARG;
      }
      fams_status_t st = fams::solve_one(h, qr, pr, o, &inf);
      if (info) info[r] = inf;
      if (st > worst) worst = st;
    }
    return worst;
  });
}

fams_status_t fams_reconstruct_flux(fams_handle_t h, const double* q, const double* p,
                                    double* flux, double* p_fv, double* imbalance) {
  if (!h || !q || !p || !flux || !fams::all_addressable({q, p, flux}) ||
      (p_fv && !fams::device_addressable(p_fv)))
    return FAMS_ERR_INVALID_ARG;
  if (h->nonsym) {
    fams::g_last_error = "the conservative flux reconstruction needs a symmetric system "
                         "(incompressible TPFA); this handle was set up as non-symmetric";
    return FAMS_ERR_INVALID_ARG;
  }
  return fams::guard([&]() -> fams_status_t {
    double imb = fams::reconstruct_flux(h, q, p, flux, p_fv);
    if (imbalance) *imbalance = imb;
    return FAMS_OK;
  });
}

fams_status_t fams_get_setup_info(fams_handle_t h, fams_setup_info_t* info) {
  if (!h || !info) return FAMS_ERR_INVALID_ARG;
  *info = h->info;
  info->device_bytes = h->alloc.live_bytes + (h->blk ? h->blk->alloc.live_bytes : 0);
  info->peak_device_bytes = h->alloc.peak_bytes + (h->blk ? h->blk->alloc.peak_bytes : 0);
  return FAMS_OK;
}

fams_status_t fams_destroy(fams_handle_t h) {
  if (!h) return FAMS_ERR_INVALID_ARG;
  return fams::guard([&]() -> fams_status_t {
    (void)hipStreamSynchronize(h->stream);
    delete h;
    return FAMS_OK;
  });
}

fams_status_t fams_get_prolongation(fams_handle_t h, int64_t* nnz, int64_t* row_ptr, int32_t* col,
                                    double* val) {
  if (!h || !nnz) return FAMS_ERR_INVALID_ARG;
  *nnz = h->p_nnz;
  if (!row_ptr && !col && !val) return FAMS_OK;
  return fams::guard([&]() -> fams_status_t {
    std::vector<int> rp(h->n + 1);
    HIPX(hipMemcpyAsync(rp.data(), h->p_rp.get(), (h->n + 1) * sizeof(int),
                        hipMemcpyDeviceToHost, h->stream));
    if (col)
      HIPX(hipMemcpyAsync(col, h->p_ci.get(), h->p_nnz * sizeof(int), hipMemcpyDeviceToHost,
                          h->stream));
    if (val)
      HIPX(hipMemcpyAsync(val, h->p_val.get(), h->p_nnz * sizeof(double), hipMemcpyDeviceToHost,
                          h->stream));
    HIPX(hipStreamSynchronize(h->stream));
    if (row_ptr)
      for (int i = 0; i <= h->n; ++i) row_ptr[i] = rp[i];
    return FAMS_OK;
  });
}

fams_status_t fams_get_coarse_matrix(fams_handle_t h, double* ac) {
  if (!h || !ac) return FAMS_ERR_INVALID_ARG;
  return fams::guard([&]() -> fams_status_t {
    HIPX(hipMemcpyAsync(ac, h->Ac.get(), sizeof(double) * h->nc * h->nc, hipMemcpyDeviceToHost,
                        h->stream));
    HIPX(hipStreamSynchronize(h->stream));
    return FAMS_OK;
  });
}

fams_status_t fams_get_ilu(fams_handle_t h, double* lu_val) {
  if (!h || !lu_val || !h->smoother) return FAMS_ERR_INVALID_ARG;
  return fams::guard([&]() -> fams_status_t {
    HIPX(hipMemcpyAsync(lu_val, h->ilu.get(), sizeof(double) * h->nnz, hipMemcpyDeviceToHost,
                        h->stream));
    HIPX(hipStreamSynchronize(h->stream));
    return FAMS_OK;
  });
}

fams_status_t fams_apply_stage(fams_handle_t h, const double* r, double* z) {
  if (!h || !r || !z || !fams::all_addressable({r, z})) return FAMS_ERR_INVALID_ARG;
  return fams::guard([&]() -> fams_status_t {
    fams::apply_stage_fp64(h, r, z);
    return FAMS_OK;
  });
}

fams_status_t fams_dense_op(int32_t op, int32_t n, const double* a, double* out) {
  if (op < 0 || op > 4 || n <= 0 || n > 65536 || !a || !out || !fams::all_addressable({a, out}))
    return FAMS_ERR_INVALID_ARG;
  return fams::guard([&]() -> fams_status_t {
    std::unique_ptr<fams_handle_s> h(new fams_handle_s());
    fams::Handle* H = h.get();
    H->stream = nullptr;
    H->alloc.stream = nullptr;
    const size_t nn = static_cast<size_t>(n) * n;
    if (op == 0) {
      HIPX(hipMemsetAsync(out, 0, nn * sizeof(double), nullptr));
      fams::dense_gemm_add(H, n, n, n, 1.0, a, n, a, n, out, n);
    } else if (op == 1) {
      FAMS_REQUIRE(fams::spd_inverse(H, a, out, n), FAMS_ERR_SINGULAR_COARSE,
                   "not positive definite");
    } else if (op == 4) {  // the packed LU factors of P A (row interchanges as in getrf)
      fams::DBuf<int> perm(&H->alloc, n);
      HIPX(hipMemcpyAsync(out, a, nn * sizeof(double), hipMemcpyDeviceToDevice, nullptr));
      fams::lu_factor(H, out, n, perm);
    } else if (op == 2) {
      fams::DBuf<double> lu(&H->alloc, nn);
      HIPX(hipMemcpyAsync(lu, a, nn * sizeof(double), hipMemcpyDeviceToDevice, nullptr));
      fams::lu_inverse(H, lu, out, n);
    } else {
      fams::DBuf<double> lu(&H->alloc, nn), e(&H->alloc, n);
      fams::DBuf<int> perm(&H->alloc, n);
      HIPX(hipMemcpyAsync(lu, a, nn * sizeof(double), hipMemcpyDeviceToDevice, nullptr));
      fams::lu_factor(H, lu, n, perm);
      std::vector<double> unit(n, 0.0);
      for (int j = 0; j < n; ++j) {
        unit[j] = 1.0;
        HIPX(hipMemcpyAsync(e, unit.data(), n * sizeof(double), hipMemcpyHostToDevice, nullptr));
        fams::lu_solve(H, lu, perm, n, e, out + static_cast<size_t>(j) * n);
        HIPX(hipStreamSynchronize(nullptr));
        unit[j] = 0.0;
      }
    }
    HIPX(hipStreamSynchronize(nullptr));
    return FAMS_OK;
  });
}

fams_status_t fams_set_profiling(fams_handle_t h, int32_t on) {
  if (!h) return FAMS_ERR_INVALID_ARG;
  return fams::guard([&]() -> fams_status_t {
    h->prof.collect();
    h->prof.on = on != 0;
    if (on) h->prof.totals.clear();
    return FAMS_OK;
  });
}

fams_status_t fams_get_kernel_stats(fams_handle_t h, int32_t max_entries, int32_t* n_entries,
                                    const char** names, double* total_ms, int64_t* launches) {
  if (!h || !n_entries) return FAMS_ERR_INVALID_ARG;
  return fams::guard([&]() -> fams_status_t {
    h->prof.collect();
    h->prof.names_cache.clear();
    for (auto& kv : h->prof.totals) h->prof.names_cache.push_back(kv.first);
    int k = 0;
    for (auto& kv : h->prof.totals) {
      if (k >= max_entries) break;
      if (names) names[k] = h->prof.names_cache[k].c_str();
      if (total_ms) total_ms[k] = kv.second.first;
      if (launches) launches[k] = kv.second.second;
      ++k;
    }
    *n_entries = static_cast<int32_t>(h->prof.totals.size());
    return FAMS_OK;
  });
}

}  // extern "C"
