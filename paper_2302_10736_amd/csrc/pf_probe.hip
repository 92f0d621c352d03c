// Streaming device copy for gfx950: the bandwidth ceiling the benchmark sets
// beside the evaluation kernels.  A copy moves its bytes with no dependent
// loads and no reductions, so at a given byte count it bounds what any
// kernel that reads half and writes half of those bytes can reach.  Not part
// of the power-flow method.
//
// Each thread copies U pairs of doubles (16-byte loads, then 16-byte
// streaming stores), U * 256 consecutive pairs per workgroup, one workgroup
// per chunk (no grid-stride loop); an odd last element is copied by the
// first thread.  U is the faster of the patterns measured on gfx950 at each
// size: 2 up to 8M pairs (128 MB each way: 4.89 us for 11.48 MB against
// 5.12 us with U = 1), 1 above (242 us for 0.77 GB each way against 265 us
// with U = 2; a grid-stride loop over at most 16384 workgroups took 284 us).

#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>

#include "pf_internal.h"

namespace pf {
namespace {

typedef double dvec2 __attribute__((ext_vector_type(2)));
constexpr int kCopyThreads = 256;
constexpr int64_t kCopyPairsU2 = int64_t(8) << 20;  // up to here two pairs per thread

template <int U>
__global__ void __launch_bounds__(kCopyThreads)
    k_stream_copy(const dvec2 *__restrict__ a, dvec2 *__restrict__ b, int64_t n2, const double *__restrict__ ta,
                  double *__restrict__ tb) {
    const int64_t first = (int64_t)blockIdx.x * (kCopyThreads * U) + threadIdx.x;
    dvec2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t i = first + (int64_t)u * kCopyThreads;
        if (i < n2) v[u] = a[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t i = first + (int64_t)u * kCopyThreads;
        if (i < n2) __builtin_nontemporal_store(v[u], b + i);
    }
    if (ta && blockIdx.x == 0 && threadIdx.x == 0) __builtin_nontemporal_store(*ta, tb);
}

template <int U>
hipError_t launch_u(const dvec2 *src, dvec2 *dst, int64_t n2, const double *ta, double *tb, hipStream_t stream) {
    const int64_t per = (int64_t)kCopyThreads * U;
    const int64_t blocks = std::max<int64_t>(1, (n2 + per - 1) / per);
    if (blocks > INT32_MAX) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_stream_copy<U>), dim3((unsigned)blocks), dim3(kCopyThreads), 0, stream, src, dst, n2, ta, tb);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stream_copy(const double *src, double *dst, int64_t n, hipStream_t stream) {
    const int64_t n2 = n / 2;
    const double *ta = (n & 1) ? src + (n - 1) : nullptr;
    double *tb = (n & 1) ? dst + (n - 1) : nullptr;
    const dvec2 *a = reinterpret_cast<const dvec2 *>(src);
    dvec2 *b = reinterpret_cast<dvec2 *>(dst);
    return n2 <= kCopyPairsU2 ? launch_u<2>(a, b, n2, ta, tb, stream) : launch_u<1>(a, b, n2, ta, tb, stream);
}

}  // namespace pf
