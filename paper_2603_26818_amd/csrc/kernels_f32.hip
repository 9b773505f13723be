// FP32 instantiation of the PFC kernels and their launchers.
#include "dispatch_impl.hpp"

namespace pfc {
PFC_INSTANTIATE(float)
}  // namespace pfc
