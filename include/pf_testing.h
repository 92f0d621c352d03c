/*
 * pf_testing.h -- measurement and testing aids exported by libpf.so beside
 * the C ABI of pf.h.  Neither is part of the power-flow method; benchmarks
 * and tests use them.  Same conventions as pf.h (status codes, device
 * pointers, pf_last_error()).
 */
#ifndef PF_TESTING_H
#define PF_TESTING_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* A streaming device copy of n doubles from src to dst (DEVICE buffers,
 * 16-byte aligned, not overlapping): 16-byte loads, then 16-byte streaming
 * stores, two pairs of doubles per thread up to 8M pairs and one above (the
 * faster pattern at each size), one workgroup per chunk of the buffers.  A
 * copy moves its bytes with no dependent loads, so at
 * a given byte count it is the practical bandwidth ceiling for a kernel that
 * reads half and writes half of those bytes; the benchmark times it beside
 * the evaluation kernels.  One launch on `stream`.  Errors: PF_EINVAL
 * (n < 0, NULL, misaligned or overlapping buffers), PF_EHIP. */
int pf_stream_copy(const double *src, double *dst, int64_t n, void *stream);

/* The next n device allocations made by the library (pf_build_pattern,
 * pf_set_schedule) fail as if the device were out of memory, so that tests
 * can check the failure paths: the call returns PF_ENOMEM and leaves any
 * existing handle as it was.  n = 0 clears the count.  Process-wide.
 * Errors: PF_EINVAL for n < 0. */
int pf_debug_fail_allocs(int32_t n);

#ifdef __cplusplus
}
#endif

#endif /* PF_TESTING_H */
