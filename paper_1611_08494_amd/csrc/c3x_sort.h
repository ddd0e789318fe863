// c3x_sort.h -- radix sort and scan entry points (device buffers, stream-ordered).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace c3x {

// Workspace for radix_sort_pairs over n elements.
size_t radix_ws_bytes(int64_t n);
// Stable LSD sort of (keys, vals) on the low nbits bits. The sorted data end
// up in (keys, vals) if *in_tmp == 0 on return, else in (ktmp, vtmp). With
// vals_are_index the values are the elements' own indices 0..n-1 and vals
// need not hold them (it is still the buffer the passes use).
// fail: a device word the caller has cleared. Given one, inputs above 32M
// elements take the one-sweep schedule, whose bounded look-back sets *fail
// to non-zero when it gives up: the order is then wrong and the inputs are
// overwritten, so the caller, which must read the word at its next
// synchronisation, redoes its work with fail = nullptr (the table schedule,
// which never gives up).
hipError_t radix_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *ktmp, uint32_t *vtmp,
                            int64_t n, int nbits, void *ws, hipStream_t s, int *in_tmp,
                            bool vals_are_index = false, uint32_t *fail = nullptr);
// The same, ordering by key bits [lo_bit, nbits) only (stable: keys equal
// in those bits keep their order).
hipError_t radix_sort_pairs_bits(uint32_t *keys, uint32_t *vals, uint32_t *ktmp, uint32_t *vtmp,
                                 int64_t n, int lo_bit, int nbits, void *ws, hipStream_t s,
                                 int *in_tmp, bool vals_are_index = false,
                                 uint32_t *fail = nullptr);

size_t scan_ws_bytes(int64_t n);
// Exclusive scans; *total (device, may be NULL) receives the sum. The
// 64-bit scan reads in[k * stride] & mask (counts inside larger records,
// flag bits masked off).
hipError_t scan_u32_to_i64(const uint32_t *in, int64_t stride, uint32_t mask, int64_t *out,
                           int64_t n, int64_t *total, void *ws, hipStream_t s);
hipError_t scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total, void *ws,
                    hipStream_t s);

}  // namespace c3x
