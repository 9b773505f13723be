// FP64 instantiation of the PFC kernels and their launchers.
#include "dispatch_impl.hpp"

namespace pfc {
PFC_INSTANTIATE(double)

__global__ void accumulate_kernel(const double *partial, int np, double coef, double *acc)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < np; ++i) s += partial[i];
        acc[0] += coef * s;
    }
}

hipError_t launch_accumulate(const double *partial, int np, double coef, double *acc, hipStream_t s)
{
    hipLaunchKernelGGL(accumulate_kernel, dim3(1), dim3(64), 0, s, partial, np, coef, acc);
    return hipGetLastError();
}
}  // namespace pfc
