// Internal declarations of the F-AMS library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <functional>
#include <initializer_list>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "../../include/fams.h"

namespace fams {

// ---- errors: thrown inside the library, converted to a status at the ABI --
struct Error : std::runtime_error {
  fams_status_t status;
  Error(fams_status_t s, const std::string& m) : std::runtime_error(m), status(s) {}
};

[[noreturn]] void hip_fail(hipError_t e, const char* what, const char* file, int line);

#define HIPX(call)                                                   \
  do {                                                               \
    hipError_t e_ = (call);                                          \
    if (e_ != hipSuccess) ::fams::hip_fail(e_, #call, __FILE__, __LINE__); \
  } while (0)

#define FAMS_REQUIRE(cond, status, msg)                              \
  do {                                                               \
    if (!(cond)) throw ::fams::Error((status), (msg));               \
  } while (0)

// ---- device memory ---------------------------------------------------------
struct Allocator {
  fams_allocator_t hook{};
  bool has_hook = false;
  hipStream_t stream = nullptr;
  int64_t live_bytes = 0;
  int64_t peak_bytes = 0;
  void* alloc(size_t bytes);
  void release(void* p, size_t bytes);
};

template <class T>
class DBuf {
 public:
  DBuf() = default;
  DBuf(Allocator* a, size_t n) { reset(a, n); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept { swap(o); }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      free();
      swap(o);
    }
    return *this;
  }
  ~DBuf() { free(); }
  void reset(Allocator* a, size_t n) {
    free();
    a_ = a;
    n_ = n;
    p_ = n ? static_cast<T*>(a->alloc(n * sizeof(T))) : nullptr;
  }
  void free() {
    if (p_ && a_) a_->release(p_, n_ * sizeof(T));
    p_ = nullptr;
    n_ = 0;
  }
  T* get() const { return p_; }
  operator T*() const { return p_; }
  size_t size() const { return n_; }

 private:
  void swap(DBuf& o) {
    std::swap(a_, o.a_);
    std::swap(p_, o.p_);
    std::swap(n_, o.n_);
  }
  Allocator* a_ = nullptr;
  T* p_ = nullptr;
  size_t n_ = 0;
};

// ---- per-kernel profiling with HIP events ----------------------------------
struct Prof {
  bool on = false;
  hipStream_t stream = nullptr;
  struct Pending {
    std::string name;
    hipEvent_t a, b;
    hipStream_t s;
  };
  std::vector<Pending> pending;
  std::map<std::string, std::pair<double, int64_t>> totals;
  std::vector<std::string> names_cache;
  // events around one launch on stream s (the handle's stream if null)
  int begin(const char* name, hipStream_t s = nullptr);
  void end(int token);
  void collect();  // synchronises the stream, folds pending events into totals
  ~Prof();
};

#define LAUNCH_ON(H, STREAM, NAME, KERNEL, GRID, BLOCK, SHMEM, ...)                \
  do {                                                                            \
    hipStream_t st_ = (STREAM);                                                   \
    int tok_ = (H)->prof.begin(NAME, st_);                                        \
    hipLaunchKernelGGL(KERNEL, dim3(GRID), dim3(BLOCK), SHMEM, st_, __VA_ARGS__);  \
    HIPX(hipGetLastError());                                                      \
    (H)->prof.end(tok_);                                                          \
  } while (0)
#define LAUNCH(H, NAME, KERNEL, GRID, BLOCK, SHMEM, ...) \
  LAUNCH_ON(H, (H)->stream, NAME, KERNEL, GRID, BLOCK, SHMEM, __VA_ARGS__)

// Auxiliary streams (default priority) for independent launches that may
// run side by side; see Fork.
constexpr int kAuxStreams = 3;
struct AuxStreams {
  hipStream_t s[kAuxStreams] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kAuxStreams] = {};
  hipEvent_t step[2] = {};  // free for one user's step-by-step hand-offs
  ~AuxStreams();
};

// Medium of unknown i: 0 matrix (i < nm), 1 fracture, 2 well (i >= nwb, the
// first well row n - nw)
__host__ __device__ __forceinline__ int medium_of(int i, int nm, int nwb) {
  return i < nm ? 0 : (i < nwb ? 1 : 2);
}

// Workgroups are dealt to the eight XCDs in turn (each with its own L2).  A
// grid padded to a multiple of eight (xcd_grid) and indexed by xcd_block
// gives XCD x the contiguous x-th eighth of the work, taken in order: for
// row-wise kernels whose rows share gathered data with nearby rows.
constexpr int kXcd = 8;

__device__ __forceinline__ int64_t xcd_block() {
  const int64_t per = gridDim.x / kXcd;
  return static_cast<int64_t>(blockIdx.x % kXcd) * per + blockIdx.x / kXcd;
}

inline unsigned xcd_grid(int64_t blocks) {
  return static_cast<unsigned>((blocks + kXcd - 1) / kXcd * kXcd);
}

// Visiting order of the rows of a lock-step sparse product.  When the first
// nm rows form a 3D grid in natural order (row = x + sy * y + sy * ny * z),
// they are visited in slabs of yb grid lines, each slab marched along z: the
// z neighbours a row gathers were then read yb * sy rows earlier (one slab
// plane, ~1 MB of a 32-wide FP64 block vector) and are still in the XCD's
// L2, where natural order re-reads them from HBM a whole grid plane later.
// The remaining rows, and all rows when sy == 0, keep natural order.  Any
// order gives the same results: each row is computed on its own.
// A sparse matrix in fixed width (the lock-step products): 8 (column,
// value) slots per row in CSR order, padded with (the row's first column,
// 0), and each row's
// CSR position and count of the entries beyond them; the values in FP64 and,
// for the precision form, FP32.  Built from the CSR arrays on first use.
struct EllMat {
  DBuf<int> col, ovf;
  DBuf<double> val;
  DBuf<float> val32;
  void clear() {
    col.free();
    ovf.free();
    val.free();
    val32.free();
  }
};

struct RowTiling {
  int nm = 0, sy = 0, ny = 0, nz = 0, yb = 0;
};

__device__ __forceinline__ int tiled_row(const RowTiling& t, int v) {
  if (t.sy == 0 || v >= t.nm) return v;
  const unsigned nx = t.sy, full = static_cast<unsigned>(t.yb) * nx * t.nz;
  const unsigned u = v, slab = u / full, rem = u - slab * full;
  const unsigned hs = min(static_cast<unsigned>(t.yb), t.ny - slab * t.yb);
  const unsigned plane = hs * nx, z = rem / plane, r2 = rem - z * plane;
  const unsigned yl = r2 / nx, x = r2 - yl * nx;
  return static_cast<int>(x + nx * (slab * t.yb + yl) + nx * t.ny * z);
}

// the handle's work-ticket words: the one-launch sweeps use the first two;
// the lock-step sweeps one counter per XCD class and direction, each on a
// cache line of its own, from kTicketBlock on
constexpr int kTicketStride = 32;
constexpr int kTicketBlock = kTicketStride;
constexpr int kTicketInts = kTicketBlock + 2 * kXcd * kTicketStride;

inline unsigned blocks_for(int64_t n, int threads) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  return static_cast<unsigned>(b);
}

// ---- level-scheduled triangular structure ---------------------------------
struct Levels {
  std::vector<int> ptr;  // host: row ranges per level in `rows`
  DBuf<int> rows;        // device: rows grouped by level, ascending within level
  DBuf<int> chunk;       // device: chunk boundaries (<= 256 rows, inside one level)
  int nchunks = 0;
  DBuf<int> bchunk;      // device: chunks of the lock-step sweeps (<= 64 rows, one level)
  int nbchunks = 0;
  DBuf<int> bchunk32;    // the same with <= 32 rows (groups of 32 right-hand sides)
  int nbchunks32 = 0;
  int count() const { return ptr.empty() ? 0 : static_cast<int>(ptr.size()) - 1; }
};

// Schedule of one triangular sweep by row ranges: rows [r*S, (r+1)*S) form
// range r; `rows` lists each range's rows grouped by dependency level
// (ascending level, then row); segment s = rows[seg[s] .. seg[s+1]) is one
// level of one range, and range r owns segments [segbase[r], segbase[r+1]).
// For the sweep kernels every position t of `rows` also carries its row's
// dependencies in sweep order: the first kEll in ELL form (ecol[t*kEll+k],
// -1 past the end, with the factor entry's CSR position epos), the count
// ecnt[t] and the first CSR position ep0[t] for the rest; the factor values
// are gathered per precision (evalN, ediagN) when the factors are known.
constexpr int kEll = 8;
struct Ranges {
  int S = 0, nranges = 0, max_segs = 0;
  DBuf<int> rows, seg, segbase;
  DBuf<int> ecol, epos, ecnt, ep0;
  DBuf<double> eval64, ediag64;
  DBuf<float> eval32, ediag32;
};

// Host phase timer: with FAMS_SETUP_TIMING set, mark() synchronises the
// stream and prints the time since the previous mark (diagnostics only).
struct PhaseTimer {
  hipStream_t stream;
  bool on;
  double t_last;
  explicit PhaseTimer(hipStream_t s);
  void mark(const char* what);
};

// ---- the handle ------------------------------------------------------------
struct Handle {
  Allocator alloc;
  hipStream_t stream = nullptr;
  Prof prof;
  AuxStreams aux;

  // options
  int variant = FAMS_DECOUPLED;
  int precision = FAMS_PREC_FP64;
  double alpha = 0.0;
  int64_t merge_cap = 4096;
  int smoother = 1;
  int restriction = 0;  // fams_restriction_t
  bool nonsym = false;  // A may be non-symmetric: LU local solves, pivoted coarse inverse

  // sizes
  int n = 0, nm = 0, nc = 0;
  int nw = 0;  // wells: the last nw unknowns (a third medium, always coarse nodes)
  int64_t nnz = 0;

  // fine system (int32 indices)
  DBuf<int> rp, ci, diag;
  DBuf<double> val;
  DBuf<float> val32;
  DBuf<int> primal, vertex;
  DBuf<int8_t> wb;           // wirebasket class of every cell
  DBuf<double> val_basis;    // the values of A the basis functions were computed from

  // prolongation / restriction (CSR)
  int64_t p_nnz = 0;
  DBuf<int> p_rp, p_ci, r_rp, r_ci;
  DBuf<double> p_val, r_val;
  DBuf<float> p_val32, r_val32;

  // coarse system: dense column-major A_c and its inverse; A P (CSR, rows in
  // A's order, columns unsorted), shared by A_c = R (A P) and the FV operator
  DBuf<double> Ac, Ainv;
  int ap_state = 0;  // 0 not built, 1 built, -1 a row exceeded the hash capacity
  DBuf<int64_t> ap_rp;
  DBuf<int> ap_ci;
  DBuf<double> ap_val;

  // ILU(0): factors in A's slots, level schedules of the two sweeps
  DBuf<double> ilu;
  DBuf<float> ilu32;
  Levels lvl_lo, lvl_up;
  Ranges rng_lo, rng_up;
  DBuf<double> sweep_in64;  // a sweep's input gathered into sweep order
  DBuf<float> sweep_in32;
  DBuf<int> ilu_ticket;  // work tickets of the two sweeps
  DBuf<int> sweep_err;   // set when a bounded wait in a sweep gives up
  unsigned long long wait_ticks = 0;  // bound of one wait, device wall-clock ticks
  int64_t lds_bytes = 0;              // dynamic LDS budget of the local block solves
  int64_t lds_hw_bytes = 0;           // dynamic LDS per workgroup the device allows

  // finite-volume stage (built lazily by fams_reconstruct_flux)
  bool fv_ready = false;
  DBuf<double> Afv, Afv_lu;
  DBuf<int> Afv_perm;
  DBuf<int> lu_flags;  // chunk flags of the dataflow LU solve (2 per 64 rows), and
  DBuf<int> lu_err;    // its error word
  int lu_epoch = 0;
  int lu_flag_n = 0;
  DBuf<int> fv_order, fv_ptr;  // cells grouped by primal block
  int fv_max_block = 0;

  // scratch of the iteration
  DBuf<double> wk;      // FP64 work vectors
  DBuf<float> wk32;     // FP32 work vectors (MIXED)
  DBuf<double> red;     // reduction partials
  DBuf<double> hred;    // small host-readable results
  DBuf<double> gpart;   // partial sums of the coarse matrix-vector product
  size_t wk_vectors = 0;

  // lock-step solves of several right-hand sides (block.hip): K values per
  // row in every block vector, m = the GMRES restart the space was sized for
  DBuf<double> bwk;     // FP64 block vectors
  DBuf<float> bwk32;    // FP32 block vectors of the precision-form stage
  DBuf<double> bred;    // reduction partials
  DBuf<double> bsmall;  // per-right-hand-side GMRES state and scalars
  DBuf<double> bpart;   // partial sums of the coarse block product
  int bK = 0, bm = 0;
  RowTiling tiling;     // visiting order of the lock-step products with A
  bool tiling_known = false;
  // A and P in fixed width for the lock-step products
  EllMat ell, pell;

  fams_setup_info_t info{};

  // per-medium smoothing stage (smoother 2): a handle of its own holding
  // A without the couplings between the media and its ILU(0) factors, and
  // the stage's correction vector
  std::unique_ptr<Handle> blk;
  DBuf<double> blk_x;
  DBuf<float> blk_x32;
};

// Fork-join of independent launches: next() hands out the handle's stream
// and then the auxiliary streams in turn, each ordered after the work the
// handle's stream held when the Fork was made; join() (also on destruction,
// where errors are ignored) makes the handle's stream wait for all of them.
class Fork {
 public:
  explicit Fork(Handle* h);
  hipStream_t next();
  void join();
  ~Fork();

 private:
  Handle* h_;
  int k_ = 0;
  bool used_[kAuxStreams] = {};
  bool joined_ = false;
};

// api.hip: pointer checks of caller arrays, and the error mapping of the C ABI
// (exceptions become a status and the thread's last error message)
bool device_addressable(const void* p);
bool all_addressable(std::initializer_list<const void*> ps);
fams_status_t guarded(const std::function<fams_status_t()>& f);

// dynamic LDS budget of one workgroup on this device (bytes, <= 160 KiB), and
// raising a kernel's dynamic LDS limit to `bytes` (api.hip)
int64_t lds_budget(Handle* h);
int64_t lds_hw_budget(Handle* h);
void allow_lds(const void* kernel, size_t bytes);
// per-block phase ticks of one launch (kTickSlots entries a block) to stderr:
// [0] start, [1] assembled, [2] factored, [3] normalised, [4] end,
// [5] n << 32 | b, [6] columns << 32 | mode, [8..12] blocked-factor phases
constexpr int kTickSlots = 16;
void print_block_timing(const unsigned long long* dev, int nb, int first);

// ---- launchers implemented in the .hip files --------------------------------
// prims.hip (rocPRIM)
void sort_pairs_i32(Handle* h, const int* keys_in, int* keys_out, const int* vals_in,
                    int* vals_out, int64_t n, int key_bits);
void exclusive_scan_i32(Handle* h, const int* in, int* out, int64_t n);
void exclusive_scan_i64(Handle* h, const int64_t* in, int64_t* out, int64_t n);

// setup.hip
void build_prolongation(Handle* h, const int8_t* wb);
// dense.hip
// the MSFV / MSMIX restriction in place of R = P^T (setup.hip)
void build_restriction(Handle* h);
void build_coarse_operator(Handle* h, const int* R_rp, const int* R_ci, const double* R_val,
                           int rows, double* out);
void lu_inverse(Handle* h, double* a, double* inv, int n);
void lu_factor(Handle* h, double* a, int n, int* perm);
bool spd_inverse(Handle* h, const double* a, double* inv, int n);
void lu_solve(Handle* h, const double* lu, const int* perm, int n, const double* b, double* x);
int lu_solve_limit();
// bound of one dataflow wait (device wall-clock ticks)
unsigned long long wait_limit(Handle* h);
void dense_gemm_add(Handle* h, int m, int p, int k, double alpha, const double* A, int lda,
                    const double* B, int ldb, double* C, int ldc);
void coarse_apply(Handle* h, const double* inv, int nc, const double* x, double* y, double* part);
// ilu.hip
void build_ilu(Handle* h);
// the per-medium smoothing stage's handle (smoother 2)
void build_block_smoother(Handle* h);
template <class T>
void ilu_apply(Handle* h, const T* lu, const T* b, T* x, T* y);
// the same for K right-hand sides in lock-step, vectors interleaved x[i * K + r]
template <class T, int K>
void ilu_apply_block(Handle* h, const T* lu, const T* b, T* x, T* y,
                     const T* add = nullptr, double* sum = nullptr);
// solve.hip
fams_status_t solve_one(Handle* h, const double* q, double* p, const fams_solve_opts_t* o,
                        fams_info_t* info);
// block.hip: nrhs right-hand sides (column-major) in lock-step groups
fams_status_t solve_block(Handle* h, const double* q, double* p, int nrhs,
                          const fams_solve_opts_t* o, fams_info_t* info);
void apply_stage_fp64(Handle* h, const double* r, double* z);
// the stage's scratch in a caller-provided region: bytes needed, and the
// stage run with its scratch there (solve.hip)
size_t stage_scratch_bytes(Handle* h);
void apply_stage_in(Handle* h, void* base, const double* r, double* z);
// noalloc.hip: the stage with its scratch in the library's static device array
void apply_stage_noalloc(Handle* h, const double* r, double* z);
size_t noalloc_scratch_capacity();
void ensure_workspace(Handle* h, int restart);
// flux.hip
double reconstruct_flux(Handle* h, const double* q, const double* p, double* flux,
                        double* p_fv);

// small helpers (solve.hip)
double dev_dot(Handle* h, const double* a, const double* b, int64_t n);
void dev_copy_d(Handle* h, double* dst, const double* src, int64_t n);

}  // namespace fams

// the opaque handle of the C ABI is the library's Handle
struct fams_handle_s : fams::Handle {};
