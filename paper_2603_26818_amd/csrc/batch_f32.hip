// FP32 instantiation of the batched persistent kernel and its launch helpers.
#include "batch.hpp"
#include "launch.hpp"

namespace pfc {
static_assert(kBatchThreads == kBatchThreadsHost, "thread count");

__shared__ cx<float> batch_lds_f32[kBatchLdsElems];
template <>
__device__ __forceinline__ cx<float> *batch_lds<float>()
{
    return batch_lds_f32;
}

template <typename T>
hipError_t launch_batch(const BatchArgs<T> &a, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((batch_kernel<T>), dim3(grid), dim3(kBatchThreads), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t batch_blocks_per_cu(int *blocks)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, batch_kernel<T>, kBatchThreads, 0);
}

template hipError_t launch_batch<float>(const BatchArgs<float> &, int, hipStream_t);
template hipError_t batch_blocks_per_cu<float>(int *);

bool batch_tiles(int n0, int M, int vx, int vy, int vc, bool f64, int *x_rows, int *c_rows, int *y_pencils)
{
    if (vx < 0 || vy < 0 || vc < 0 || vx >= batch_candidates(n0, M, 0) || vy >= batch_candidates(n0, M, 1) ||
        vc >= batch_candidates(n0, M, 2))
        return false;
    bool ok = true;
    auto xr = [&](int m) {
        switch (m) {
#define PFC_XCASE(MM)                                                                                   \
    case MM:                                                                                            \
        with_plan<typename XFwdCands<MM>::type>(vx, [&](auto p) { *x_rows = BRows<decltype(p)>::value; return 0; }); \
        with_plan<typename XInvCands<MM>::type>(vc, [&](auto p) { *c_rows = BRows<decltype(p)>::value; return 0; }); \
        break;
            PFC_XCASE(16) PFC_XCASE(32) PFC_XCASE(64) PFC_XCASE(128) PFC_XCASE(256) PFC_XCASE(512)
#undef PFC_XCASE
        default: ok = false;
        }
    };
    auto yr = [&](int l) {
        switch (l) {
#define PFC_YCASE(LL)                                                                                   \
    case LL:                                                                                            \
        with_plan<typename LastCands<LL>::type>(vy, [&](auto p) {                                         \
            using P0 = decltype(p);                                                                     \
            *y_pencils = f64 ? kBatchThreads / SpreadIf<P0, PencilTile<double, LL>::E>::Tp               \
                             : kBatchThreads / SpreadIf<P0, PencilTile<float, LL>::E>::Tp;               \
            return 0;                                                                                   \
        });                                                                                             \
        break;
            PFC_YCASE(32) PFC_YCASE(64) PFC_YCASE(128) PFC_YCASE(256) PFC_YCASE(512) PFC_YCASE(1024)
#undef PFC_YCASE
        default: ok = false;
        }
    };
    xr(M);
    yr(n0);
    return ok;
}

int batch_candidates(int n0, int M, int pass)
{
    const int len = pass == 1 ? n0 : M;
    switch (len) {
#define PFC_CCASE(LL)                                                                                   \
    case LL:                                                                                            \
        return pass == 0 ? XFwdCands<LL>::type::size : pass == 1 ? LastCands<LL>::type::size : XInvCands<LL>::type::size;
        PFC_CCASE(16) PFC_CCASE(32) PFC_CCASE(64) PFC_CCASE(128) PFC_CCASE(256) PFC_CCASE(512) PFC_CCASE(1024)
#undef PFC_CCASE
    default: return 0;
    }
}
}  // namespace pfc
