// api_internal.hpp -- library-internal calls between pfc_api.cpp and the allocation-free step
// (noalloc.hip).  Not part of the C ABI.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "../../include/pfc.h"

namespace pfc_internal {

// Bytes of the plan's twiddle tables (rounded up to 256) and of one native spectrum.
size_t table_bytes(const pfc_plan *p);
size_t spectrum_bytes(const pfc_plan *p);
// The plan's device ordinal and its process-unique id.
int plan_device(const pfc_plan *p);
uint64_t plan_id(const pfc_plan *p);
// Records a detail string for pfc_last_error() and returns st.
pfc_status report(pfc_status st, const char *msg);
// Checks psi, state and nsteps as pfc_step does (the plan's own workspace is not needed).
pfc_status check_step_args(const pfc_plan *p, const void *psi, const void *state, int64_t nsteps);
// Queues a copy of the plan's twiddle tables to the device address `tables` on `stream` (the
// plan holds the host copy; it must stay alive until the copy has run).
pfc_status upload_tables(pfc_plan *p, void *tables, void *stream);
// pfc_step with the twiddle tables at `tables` and the scratch spectrum at `spectrum` (device
// addresses on the plan's device, 256-byte aligned) instead of the plan's workspace.
pfc_status step_with_buffers(pfc_plan *p, void *psi, void *state, int64_t nsteps, void *stream, void *tables,
                             void *spectrum);

}  // namespace pfc_internal
