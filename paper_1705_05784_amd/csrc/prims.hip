// Stable sorts and prefix sums used by the setup's bookkeeping (rocPRIM).
// Stability gives every ordering the library builds a fixed, run-independent
// order (cells ascending inside a block, fine rows ascending inside a row of
// R = P^T, rows ascending inside an ILU level).
#include <cstring>

#include <rocprim/rocprim.hpp>

#include "internal.hpp"

namespace fams {

void sort_pairs_i32(Handle* h, const int* keys_in, int* keys_out, const int* vals_in,
                    int* vals_out, int64_t n, int key_bits) {
  if (n <= 0) return;
  FAMS_REQUIRE(n < (int64_t(1) << 31), FAMS_ERR_CAPACITY, "sort size");
  size_t tmp = 0;
  HIPX(rocprim::radix_sort_pairs(nullptr, tmp, keys_in, keys_out, vals_in, vals_out,
                                 static_cast<unsigned>(n), 0, key_bits, h->stream));
  DBuf<char> t(&h->alloc, tmp ? tmp : 1);
  HIPX(rocprim::radix_sort_pairs(t.get(), tmp, keys_in, keys_out, vals_in, vals_out,
                                 static_cast<unsigned>(n), 0, key_bits, h->stream));
}

void exclusive_scan_i32(Handle* h, const int* in, int* out, int64_t n) {
  if (n <= 0) return;
  size_t tmp = 0;
  HIPX(rocprim::exclusive_scan(nullptr, tmp, in, out, 0, static_cast<size_t>(n),
                               rocprim::plus<int>(), h->stream));
  DBuf<char> t(&h->alloc, tmp ? tmp : 1);
  HIPX(rocprim::exclusive_scan(t.get(), tmp, in, out, 0, static_cast<size_t>(n),
                               rocprim::plus<int>(), h->stream));
}

void exclusive_scan_i64(Handle* h, const int64_t* in, int64_t* out, int64_t n) {
  if (n <= 0) return;
  size_t tmp = 0;
  HIPX(rocprim::exclusive_scan(nullptr, tmp, in, out, int64_t(0), static_cast<size_t>(n),
                               rocprim::plus<int64_t>(), h->stream));
  DBuf<char> t(&h->alloc, tmp ? tmp : 1);
  HIPX(rocprim::exclusive_scan(t.get(), tmp, in, out, int64_t(0), static_cast<size_t>(n),
                               rocprim::plus<int64_t>(), h->stream));
}

}  // namespace fams
