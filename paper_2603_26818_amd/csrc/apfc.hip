// apfc.hip -- launchers of the complex-amplitude kernels (apfc.hpp), FP32 and FP64.
#include "apfc.hpp"
#include "apfc_launch.hpp"
#include "dispatch_impl.hpp"

namespace pfc {

constexpr int64_t kApfcCUs = 256;  // compute units of the MI355X

template <typename T>
hipError_t launch_apfc_nonlin(const cx<T> *eta, cx<T> *out, int64_t P, int nf, const ApfcTerm *terms, const int *off,
                              double c3, hipStream_t s)
{
    if (nf < 1 || nf > kApfcMaxFields) return hipErrorInvalidValue;
    // two points per thread while their LDS slots fit in 64 KB (all but FP64 with over 16 fields)
    const size_t lds2 = (size_t)nf * 2 * kApfcThreads * sizeof(cx<T>);
    if (lds2 <= 65536) {
        hipLaunchKernelGGL((apfc_nonlin_kernel<T, 2>), dim3((unsigned)cdiv(P, 2 * kApfcThreads)), dim3(kApfcThreads),
                           lds2, s, eta, out, P, nf, terms, off, (T)c3);
    } else {
        hipLaunchKernelGGL((apfc_nonlin_kernel<T, 1>), dim3((unsigned)cdiv(P, kApfcThreads)), dim3(kApfcThreads),
                           lds2 / 2, s, eta, out, P, nf, terms, off, (T)c3);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_apfc_rows(int64_t L, const cx<T> *in, cx<T> *out, int64_t nrows, int dir, double scale, bool nt,
                            const cx<T> *tw, int lt_shift, hipStream_t s)
{
    return by_length(L, [&](auto Lc) -> hipError_t {
        constexpr int LL = decltype(Lc)::value;
        if constexpr (LL < 4) {
            return hipErrorInvalidValue;
        } else {
            using PL = typename DefaultPlan<LL>::type;
            constexpr int ROWS = XRows<PL>::value;
            const dim3 grid((unsigned)cdiv(nrows, ROWS)), block(ROWS * PL::Tp);
            return with_nt(nt, [&](auto ntc) -> hipError_t {
                constexpr bool NT = decltype(ntc)::value;
                if (dir < 0)
                    hipLaunchKernelGGL((apfc_row_kernel<T, PL, ROWS, -1, NT>), grid, block, 0, s, in, out, nrows, tw,
                                       lt_shift, (T)scale);
                else
                    hipLaunchKernelGGL((apfc_row_kernel<T, PL, ROWS, +1, NT>), grid, block, 0, s, in, out, nrows, tw,
                                       lt_shift, (T)scale);
                return hipGetLastError();
            });
        }
    });
}

template <typename T>
hipError_t launch_apfc_last_step(int64_t L, int nf, ApfcStepArgs<T> a, hipStream_t s)
{
    return by_length(L, [&](auto Lc) -> hipError_t {
        constexpr int LL = decltype(Lc)::value;
        if constexpr (LL < 4) {
            return hipErrorInvalidValue;
        } else {
            using TL = PencilTile<T, LL>;
            using PL = SpreadIf<typename AxisPlan<LL>::type, TL::E>;
            auto run = [&](auto wc, auto gc, auto plc) -> hipError_t {
                constexpr int WM = decltype(wc)::value, G = decltype(gc)::value;
                using PLr = decltype(plc);
                constexpr bool PF = is_pow2c(LL) && PLr::Rmax <= 16;  // state prefetch while registers allow
                a.W = (int)(a.ncols < WM ? a.ncols : WM);
                a.tiles = cdiv(a.ncols, a.W);
                const dim3 grid((unsigned)(a.tiles * nf)), block(WM * PLr::Tp);
                hipLaunchKernelGGL((apfc_last_step_kernel<T, PLr, WM, PF, G>), grid, block, 0, s, a);
                return hipGetLastError();
            };
            // The grouped long tiles fill a CU each: with few pencil columns (2D grids) their count
            // leaves the last round of workgroups partly empty.  Half-width tiles in one LDS group
            // (still one per CU) double the count, and the rounds fill up; they take the length's
            // plain schedule (16 elements per thread, twice the threads of the spread one), whose
            // registers leave room to prefetch the state.
            if constexpr (TL::G == 2 && TL::W == 16) {
                const int64_t full = cdiv(a.ncols, TL::W) * nf;
                if (full < 4 * kApfcCUs && (full % kApfcCUs) != 0)
                    return run(std::integral_constant<int, TL::W / 2>{}, std::integral_constant<int, 1>{},
                               typename AxisPlan<LL>::type{});
            }
            return run(std::integral_constant<int, TL::W>{}, std::integral_constant<int, TL::G>{}, PL{});
        }
    });
}

#define PFC_APFC_INSTANTIATE(T)                                                                                   \
    template hipError_t launch_apfc_nonlin<T>(const cx<T> *, cx<T> *, int64_t, int, const ApfcTerm *, const int *, \
                                              double, hipStream_t);                                                \
    template hipError_t launch_apfc_rows<T>(int64_t, const cx<T> *, cx<T> *, int64_t, int, double, bool,          \
                                            const cx<T> *, int, hipStream_t);                                      \
    template hipError_t launch_apfc_last_step<T>(int64_t, int, ApfcStepArgs<T>, hipStream_t);
PFC_APFC_INSTANTIATE(float)
PFC_APFC_INSTANTIATE(double)

}  // namespace pfc
