// FP64 instantiation of the batched persistent kernel and its launch helpers.
#include "batch.hpp"
#include "launch.hpp"

namespace pfc {
static_assert(kBatchThreads == kBatchThreadsHost, "thread count");

__shared__ cx<double> batch_lds_f64[kBatchLdsElems];
template <>
__device__ __forceinline__ cx<double> *batch_lds<double>()
{
    return batch_lds_f64;
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

template hipError_t launch_batch<double>(const BatchArgs<double> &, int, hipStream_t);
template hipError_t batch_blocks_per_cu<double>(int *);
}  // namespace pfc
