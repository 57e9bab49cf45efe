// Device binary64 square root and division as the growth kernels evaluate
// them (their settings; the hard-sphere kernels' own square root on
// [2^-60, 1]), so that a host program can check them against the correctly
// rounded host results (the hard-sphere kernels rely on both being correctly
// rounded to match the CPU bit for bit; Sec. 3.3.3).
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "rsaw.h"
#include "rsaw_device.hpp"

namespace rsaw {

__global__ __launch_bounds__(256) void fp64_check_kernel(const double *a, const double *b, double *sq, double *dv,
                                                         uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double x = a[i];
        // the hard-sphere kernels' square root on its domain, else the general one
        sq[i] = (x >= 0x1p-60 && x <= 1.0) ? sqrt_unit(x) : sqrt(x);
        dv[i] = x / b[i];
    }
}

} // namespace rsaw

extern "C" rsaw_status rsaw_fp64_check(const double *d_a, const double *d_b, double *d_sqrt, double *d_div,
                                       uint64_t n, void *stream)
{
    if (n == 0) return RSAW_OK;
    if (!d_a || !d_b || !d_sqrt || !d_div) return RSAW_E_INVALID;
    const uint64_t blocks64 = (n + 255) / 256;
    const unsigned blocks = (unsigned)(blocks64 < 8192 ? blocks64 : 8192);
    hipLaunchKernelGGL(rsaw::fp64_check_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, d_a, d_b, d_sqrt,
                       d_div, n);
    return hipGetLastError() == hipSuccess ? RSAW_OK : RSAW_E_DEVICE;
}
