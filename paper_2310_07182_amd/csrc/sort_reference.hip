// rocPRIM's device radix sort behind the C entry points of pt_sortref.h (a yardstick for the
// sorted modes' own radix sort; not part of any render path).
#include <cstring>

#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>

#include "../../include/pt_sortref.h"

extern "C" int ptref_sort_workspace_bytes(uint32_t n, int end_bit, size_t* bytes) {
    if (!bytes || end_bit < 1 || end_bit > 32) return (int)hipErrorInvalidValue;
    size_t b = 0;
    const hipError_t e = rocprim::radix_sort_pairs(nullptr, b, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                                   (const uint32_t*)nullptr, (uint32_t*)nullptr, (size_t)n, 0,
                                                   end_bit);
    *bytes = b;
    return (int)e;
}

extern "C" int ptref_sort_pairs(void* workspace, size_t workspace_bytes, const uint32_t* kin, uint32_t* kout,
                                const uint32_t* vin, uint32_t* vout, uint32_t n, int end_bit, void* stream) {
    if (end_bit < 1 || end_bit > 32) return (int)hipErrorInvalidValue;
    if (n == 0) return 0;
    size_t need = 0;
    const int q = ptref_sort_workspace_bytes(n, end_bit, &need);
    if (q != 0) return q;
    if (!workspace || workspace_bytes < need || !kin || !kout || !vin || !vout) return (int)hipErrorInvalidValue;
    size_t b = workspace_bytes;
    return (int)rocprim::radix_sort_pairs(workspace, b, kin, kout, vin, vout, (size_t)n, 0, end_bit,
                                          (hipStream_t)stream);
}
