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

int step_candidates(const Geom &g, int pass)
{
    // pass ids as pfc_step_timed: 3D 0 x r2c, 1 y fwd, 2 last, 3 y inv, 4 x c2r; 2D 0 x r2c, 1 last, 2 x c2r
    const int id = (g.ndim == 3) ? pass : (pass == 0 ? 0 : pass == 1 ? 2 : pass == 2 ? 4 : -1);
    int n = 0;
    auto count = [&](auto lc, auto kind) -> hipError_t {
        constexpr int L = decltype(lc)::value;
        constexpr int K = decltype(kind)::value;
        if constexpr (K == 0) n = XFwdCands<L>::type::size;
        else if constexpr (K == 1) n = AxisCands<L>::type::size;
        else if constexpr (K == 2) n = (g.ndim == 3) ? ZCands<L>::type::size : LastCands<L>::type::size;
        else n = XInvCands<L>::type::size;
        return hipSuccess;
    };
    switch (id) {
    case 0: (void)by_length(g.M, [&](auto l) { return count(l, std::integral_constant<int, 0>{}); }); break;
    case 1:
    case 3: (void)by_length(g.n1, [&](auto l) { return count(l, std::integral_constant<int, 1>{}); }); break;
    case 2: (void)by_length(g.n0, [&](auto l) { return count(l, std::integral_constant<int, 2>{}); }); break;
    case 4: (void)by_length(g.M, [&](auto l) { return count(l, std::integral_constant<int, 3>{}); }); break;
    default: break;
    }
    return n;
}

hipError_t launch_accumulate(const double *partial, int np, double coef, double *acc, hipStream_t s)
{
    hipLaunchKernelGGL(accumulate_kernel, dim3(1), dim3(64), 0, s, partial, np, coef, acc);
    return hipGetLastError();
}
}  // namespace pfc
