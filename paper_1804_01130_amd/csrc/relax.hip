// Relaxation zones: alpha blended towards a target after the advection step (Section 3, wave
// generation and absorption, with the exponential weight of Jacobsen, Fuhrman & Fredsoe 2012).
//
// The plan holds the cells whose centres lie in a zone and their weights w, computed once on the
// host when the zones are set.  Per call, one thread per zone cell replaces alpha by
// w alpha + (1 - w) alpha_target in place.  A pure stream: 36 bytes per zone cell (index,
// weight, alpha read and written, target read), bound by HBM bandwidth.  FMA contraction is off,
// so the blend rounds operation by operation in the order written.
#include "device_common.h"
#include "internal.h"

namespace isoadv {

namespace {

__global__ __launch_bounds__(256) void k_relax_blend(const int32_t *__restrict__ cells, const double *__restrict__ w,
                                                      int64_t n, double *__restrict__ alpha,
                                                      const double *__restrict__ target) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int32_t c = __builtin_nontemporal_load(cells + i);
    const double wi = __builtin_nontemporal_load(w + i);
    const double a = __builtin_nontemporal_load(alpha + c), t = __builtin_nontemporal_load(target + c);
    __builtin_nontemporal_store(wi * a + (1.0 - wi) * t, alpha + c);
}

}  // namespace

hipError_t launch_relax_blend(const int32_t *cells, const double *w, int64_t n, double *alpha, const double *target,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_relax_blend, dim3((unsigned)blocks), dim3(256), 0, s, cells, w, n, alpha, target);
    return hipGetLastError();
}

}  // namespace isoadv
