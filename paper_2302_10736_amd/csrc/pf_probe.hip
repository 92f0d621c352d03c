// Streaming device copy for gfx950: the bandwidth ceiling the benchmark sets
// beside the evaluation kernels.  A copy moves its bytes with no dependent
// loads and no reductions, so at a given byte count it bounds what any
// kernel that reads half and writes half of those bytes can reach.  Not part
// of the power-flow method.
//
// One 16-byte load and one 16-byte streaming store per thread and step,
// grid-stride over the pairs of doubles; an odd last element is copied by
// the first thread.

#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>

#include "pf_internal.h"

namespace pf {
namespace {

typedef double dvec2 __attribute__((ext_vector_type(2)));
constexpr int kCopyThreads = 256;
constexpr int64_t kCopyMaxBlocks = 16384;

__global__ void __launch_bounds__(kCopyThreads)
    k_stream_copy(const dvec2 *__restrict__ a, dvec2 *__restrict__ b, int64_t n2, const double *__restrict__ ta,
                  double *__restrict__ tb) {
    const int64_t stride = (int64_t)gridDim.x * kCopyThreads;
    const int64_t first = (int64_t)blockIdx.x * kCopyThreads + threadIdx.x;
    for (int64_t i = first; i < n2; i += stride) __builtin_nontemporal_store(a[i], b + i);
    if (ta && first == 0) __builtin_nontemporal_store(*ta, tb);
}

}  // namespace

hipError_t launch_stream_copy(const double *src, double *dst, int64_t n, hipStream_t stream) {
    const int64_t n2 = n / 2;
    const int64_t want = (n2 + kCopyThreads - 1) / kCopyThreads;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(want, kCopyMaxBlocks));
    const double *ta = (n & 1) ? src + (n - 1) : nullptr;
    double *tb = (n & 1) ? dst + (n - 1) : nullptr;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(kCopyThreads), 0, stream,
                       reinterpret_cast<const dvec2 *>(src), reinterpret_cast<dvec2 *>(dst), n2, ta, tb);
    return hipGetLastError();
}

}  // namespace pf
