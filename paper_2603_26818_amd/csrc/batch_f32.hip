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

bool batch_tiles(int n0, int M, int *x_rows, int *c_rows, int *y_pencils)
{
    auto xr = [](int m, int *f, int *c) {
        switch (m) {
#define PFC_XCASE(MM)                                                     \
    case MM:                                                              \
        *f = BRows<typename BXFwd<MM>::type>::value;                      \
        *c = BRows<typename BXInv<MM>::type>::value;                      \
        return true;
            PFC_XCASE(16) PFC_XCASE(32) PFC_XCASE(64) PFC_XCASE(128) PFC_XCASE(256) PFC_XCASE(512)
#undef PFC_XCASE
        default: return false;
        }
    };
    auto yr = [](int l, int *w) {
        switch (l) {
#define PFC_YCASE(LL)                                                     \
    case LL:                                                              \
        *w = kBatchThreads / BLast<LL>::type::Tp;                         \
        return true;
            PFC_YCASE(32) PFC_YCASE(64) PFC_YCASE(128) PFC_YCASE(256) PFC_YCASE(512) PFC_YCASE(1024)
#undef PFC_YCASE
        default: return false;
        }
    };
    return xr(M, x_rows, c_rows) && yr(n0, y_pencils);
}
template hipError_t batch_blocks_per_cu<float>(int *);
}  // namespace pfc
