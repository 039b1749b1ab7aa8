// fams_apply_stage_noalloc: the preconditioner application of
// fams_apply_stage without any device allocation, for callers that cannot
// allocate (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).  Its scratch lives in one file-scope device array of
// kScratchBytes, which every GPU the library runs on holds until the process
// ends; its device address is looked up once per device (the array's name
// is only a host-side stand-in in host code).  Everything else the stage
// touches belongs to the handle and is allocated by fams_setup.
#include <mutex>

#include "internal.hpp"

namespace fams {
namespace {

constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on the current device (looked up with that
// device current, once per device)
void* scratch_on_current_device() {
  int dev = 0;
  HIPX(hipGetDevice(&dev));
  FAMS_REQUIRE(dev >= 0 && dev < kMaxDevices, FAMS_ERR_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPX(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    FAMS_REQUIRE(p != nullptr, FAMS_ERR_DEVICE, "no device address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

size_t noalloc_scratch_capacity() { return kScratchBytes; }

void apply_stage_noalloc(Handle* h, const double* r, double* z) {
  const size_t need = stage_scratch_bytes(h);
  FAMS_REQUIRE(need <= kScratchBytes, FAMS_ERR_CAPACITY,
               "system too large for the allocation-free stage: needs " + std::to_string(need) +
                   " bytes of scratch, the library holds " + std::to_string(kScratchBytes));
  void* base = scratch_on_current_device();
  // no per-launch timing events here: creating them is not allowed either
  const bool prof = h->prof.on;
  h->prof.on = false;
  try {
    apply_stage_in(h, base, r, z);
  } catch (...) {
    h->prof.on = prof;
    throw;
  }
  h->prof.on = prof;
}

}  // namespace fams

extern "C" fams_status_t fams_apply_stage_noalloc(fams_handle_t h, const double* r, double* z) {
  if (!h || !r || !z || !fams::all_addressable({r, z})) return FAMS_ERR_INVALID_ARG;
  return fams::guarded([&]() -> fams_status_t {
    fams::apply_stage_noalloc(h, r, z);
    return FAMS_OK;
  });
}
