/* libptsortref: the vendor library's device radix sort behind a C entry point, a yardstick
 * for the radix sort of the sorted modes (pt_sort_pairs).  Not used by any render path.
 *
 * The sorted modes of the paper's comparison (Section 5.1, Table 1) reorder each bounce's
 * rays by a 30-bit key before tracing; the time of that sort is what the reordering costs.
 * This library sorts the same (key, value) pairs with rocPRIM's device radix_sort_pairs so
 * that the benchmark can time both on one GPU.
 *
 * Status: 0 = success, else the hipError_t value of the failing call. */
#ifndef PT_SORTREF_H
#define PT_SORTREF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Device workspace bytes that ptref_sort_pairs needs for n pairs sorted by bits [0, end_bit)
 * (1 <= end_bit <= 32), written to *bytes. */
int ptref_sort_workspace_bytes(uint32_t n, int end_bit, size_t* bytes);

/* Stable sort of n (key, value) pairs by bits [0, end_bit) of the 32-bit key: kin, vin (device,
 * [n] uint32, read only) to kout, vout (device, [n] uint32, written; must not overlap the
 * inputs).  workspace: device, >= ptref_sort_workspace_bytes(n, end_bit).  stream: a
 * hipStream_t (null = the default stream).  Asynchronous on stream; the caller owns every
 * buffer. */
int ptref_sort_pairs(void* workspace, size_t workspace_bytes, const uint32_t* kin, uint32_t* kout,
                     const uint32_t* vin, uint32_t* vout, uint32_t n, int end_bit, void* stream);

#ifdef __cplusplus
}
#endif

#endif
