// batch.hpp -- persistent kernel that advances many independent 2D PFC runs of mixed sizes.
//
// One launch runs `nsteps` steps of every instance.  A step is three passes (x r2c with cube,
// y forward + update + y inverse, x c2r); each pass is a list of work items (a group of rows or a
// tile of columns of one instance), and the persistent workgroups take items round-robin.  A grid
// barrier separates passes.  Between two steps the x c2r of one step and the x r2c of the next
// touch the same rows only, so they run as one fused pass (an item: the c2r blocks of a row group,
// then the r2c blocks of the same rows, which read the fresh psi back from the L2): two barriers
// per step instead of three.  Every workgroup has NT threads; each size runs a schedule whose
// thread count per item is exactly NT, so one kernel serves all sizes.
//
// The grid barrier waits a bounded number of polls.  If the wait runs out (the workgroups are not
// all resident), it sets an error flag and every workgroup leaves the kernel at its next barrier,
// so the launch always terminates; the host reads the flag (pfc_batch_check).
#pragma once

#include "kernels.hpp"

namespace pfc {

constexpr int kBatchThreads = 512;
constexpr int kBatchMaxInst = 256;

// Schedules of the batched passes: the same candidate lists as the single-plan passes; each item
// has NT / Tp rows (x passes) or pencils (y pass).  Each instance records its candidate per pass.

template <class PL>
struct BRows {
    static constexpr int value = kBatchThreads / PL::Tp;
};

// Grid-wide barrier across the persistent workgroups (all resident).  Release: write back this
// XCD's L2 before arriving; acquire: invalidate it after the wait, so stores of every workgroup
// before the barrier are visible to loads of every workgroup after it.  Returns false (for the
// whole workgroup) if an error flag is set or the wait timed out.
__device__ __forceinline__ bool grid_sync(BatchCtl *ctl, unsigned nblocks, unsigned long long max_polls)
{
    __shared__ int ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        int good = 1;
        if (__hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            good = 0;
        } else {
            const unsigned g = __hip_atomic_load(&ctl->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const unsigned a = __hip_atomic_fetch_add(&ctl->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (a + 1 == nblocks) {
                __hip_atomic_store(&ctl->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(&ctl->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                unsigned long long polls = 0;
                while (__hip_atomic_load(&ctl->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                    if (__hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                        good = 0;
                        break;
                    }
                    if (++polls > max_polls) {
                        __hip_atomic_store(&ctl->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        good = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        ok = good;
    }
    __syncthreads();
    return ok != 0;
}

// instance owning global item k of a pass (items of instance i are [begin_i, begin_{i+1}))
template <typename T, int PASS>
__device__ __forceinline__ int find_inst(const BatchArgs<T> &a, int k)
{
    int i = 0;
    while (i + 1 < a.ninst) {
        const BatchInst<T> &n = a.inst[i + 1];
        const int b = PASS == 0 ? n.x_begin : PASS == 1 ? n.y_begin : PASS == 2 ? n.c_begin : n.f_begin;
        if (k < b) break;
        ++i;
    }
    return i;
}

// The per-size pass bodies are separate (non-inlined) functions: inlined into one kernel, the
// schedules of all sizes interfere in register allocation and spill heavily.  They reach LDS
// through a file-scope __shared__ array (defined by the including translation unit, one dtype per
// unit), so their LDS accesses stay ds_* instructions.
template <typename T>
__device__ __forceinline__ cx<T> *batch_lds();

template <typename T, class PL>
__device__ __noinline__ void batch_x_fwd(const BatchInst<T> *in, int item, const cx<T> *tw, int lt_shift)
{
    x_r2c_block<T, PL, BRows<PL>::value, true>(in->psi, in->scratch, in->n0, tw, lt_shift, item, batch_lds<T>(),
                                              row_pack(in->M));
}

// Lengths whose single-plan step uses a spread tile (PencilTile) use the same tile here, so that
// each instance computes exactly what its own plan computes.
template <typename T, class PL0>
__device__ __noinline__ void batch_y_step(const BatchInst<T> *in, int item, const cx<T> *tw, int lt_shift)
{
    using TL = PencilTile<T, PL0::L>;
    using PL = SpreadIf<PL0, TL::E>;
    constexpr int WM = kBatchThreads / PL::Tp;
    static_assert(TL::G == 1 || WM == TL::W, "spread tile must fill the batched workgroup");
    LastAxisArgs<T> la{};
    la.src = in->scratch;
    la.dst = in->scratch;
    la.dst2 = nullptr;
    la.state = in->state;
    la.nrows = 1;
    la.M = in->M;
    la.W = in->W;
    la.tiles_per_row = in->tiles;
    la.tw = tw;
    la.lt_shift = lt_shift;
    la.mp = in->mp;
    la.pk = row_pack(in->M);
    last_axis_block<T, PL, WM, LA_STEP, TL::PF, ORD_TILE, false, TL::G>(la, item, batch_lds<T>());
}

// x c2r of a row group fused with the cube and x r2c of the next step (the single-plan step's
// fused kernel body, with this kernel's thread count): rows [item f_rows, (item + 1) f_rows)
template <typename T, class PLI, class PLF>
__device__ __noinline__ void batch_x_fused(const BatchInst<T> *in, int item, const cx<T> *tw, int lt_shift)
{
    x_c2r_r2c_block<T, PLI, PLF, kBatchThreads>(in->scratch, in->scratch, in->n0, tw, lt_shift, in->sc, item,
                                                batch_lds<T>(), row_pack(in->M));
}

template <typename T, class PL>
__device__ __noinline__ void batch_x_inv(const BatchInst<T> *in, int item, const cx<T> *tw, int lt_shift)
{
    AdjEpi<T> ea{};
    x_c2r_block<T, PL, BRows<PL>::value, EPI_PLAIN>(in->scratch, in->psi, in->n0, tw, lt_shift, in->sc, ea, item,
                                                     batch_lds<T>(), row_pack(in->M));
}

// supported lengths: x 32..1024 (M = 16..512), y 32..1024
#define PFC_BCASE(LEN, CANDS, FN, VAR)                                                                       \
    case LEN:                                                                                                \
        with_plan<typename CANDS<LEN>::type>(VAR, [&](auto plc) {                                            \
            FN<T, decltype(plc)>(in, item, tw, lt);                                                          \
            return 0;                                                                                        \
        });                                                                                                  \
        break;

template <typename T>
__device__ __forceinline__ void batch_pass(int pass, const BatchInst<T> *in, int item, const cx<T> *tw, int lt)
{
    if (pass == 0) {
        switch (in->M) {
            PFC_BCASE(16, XFwdCands, batch_x_fwd, in->vx)
            PFC_BCASE(32, XFwdCands, batch_x_fwd, in->vx)
            PFC_BCASE(64, XFwdCands, batch_x_fwd, in->vx)
            PFC_BCASE(128, XFwdCands, batch_x_fwd, in->vx)
            PFC_BCASE(256, XFwdCands, batch_x_fwd, in->vx)
            PFC_BCASE(512, XFwdCands, batch_x_fwd, in->vx)
        default: break;
        }
    } else if (pass == 1) {
        switch (in->n0) {
            PFC_BCASE(32, LastCands, batch_y_step, in->vy)
            PFC_BCASE(64, LastCands, batch_y_step, in->vy)
            PFC_BCASE(128, LastCands, batch_y_step, in->vy)
            PFC_BCASE(256, LastCands, batch_y_step, in->vy)
            PFC_BCASE(512, LastCands, batch_y_step, in->vy)
            PFC_BCASE(1024, LastCands, batch_y_step, in->vy)
        default: break;
        }
    } else {
        switch (in->M) {
            PFC_BCASE(16, XInvCands, batch_x_inv, in->vc)
            PFC_BCASE(32, XInvCands, batch_x_inv, in->vc)
            PFC_BCASE(64, XInvCands, batch_x_inv, in->vc)
            PFC_BCASE(128, XInvCands, batch_x_inv, in->vc)
            PFC_BCASE(256, XInvCands, batch_x_inv, in->vc)
            PFC_BCASE(512, XInvCands, batch_x_inv, in->vc)
        default: break;
        }
    }
}
#undef PFC_BCASE

// LDS needed by the largest schedule: NT * Rmax complex values (Rmax <= 16).
constexpr int kBatchLdsElems = kBatchThreads * 16;

// Fused item between two steps: x c2r of rows [item f_rows, (item + 1) f_rows), the field kept in
// LDS, cube and x r2c of the same rows (f_rows is XFused<..>::R of the two schedules).
#define PFC_FCASE(LEN)                                                                                     \
    case LEN:                                                                                              \
        with_plan<typename XInvCands<LEN>::type>(in->vc, [&](auto pi) {                                    \
            return with_plan<typename XFwdCands<LEN>::type>(in->vx, [&](auto pf) {                         \
                batch_x_fused<T, decltype(pi), decltype(pf)>(in, item, tw, lt);                            \
                return 0;                                                                                  \
            });                                                                                            \
        });                                                                                                \
        break;
template <typename T>
__device__ __forceinline__ void batch_fused(const BatchInst<T> *in, int item, const cx<T> *tw, int lt)
{
    switch (in->M) {
        PFC_FCASE(16) PFC_FCASE(32) PFC_FCASE(64) PFC_FCASE(128) PFC_FCASE(256) PFC_FCASE(512)
    default: break;
    }
}
#undef PFC_FCASE

// 2 workgroups of kBatchThreads per CU (4 waves per SIMD).
template <typename T>
__global__ __launch_bounds__(kBatchThreads, 4) void batch_kernel(BatchArgs<T> a)
{
    const unsigned G = gridDim.x;
    for (int64_t step = 0; step < a.nsteps; ++step) {
        // pass 0: x r2c (first step only; later steps get it from the fused pass), 1: y, then
        // 2: x c2r after the last step, 3: fused x c2r + next step's x r2c otherwise
        for (int pass = (step == 0 ? 0 : 1); pass < 3; ++pass) {
            const int kind = (pass == 2 && step + 1 < a.nsteps) ? 3 : pass;
            const int total = kind == 0 ? a.x_total : kind == 1 ? a.y_total : kind == 2 ? a.c_total : a.f_total;
            for (int k = blockIdx.x; k < total; k += G) {
                const int i = kind == 0 ? find_inst<T, 0>(a, k) : kind == 1 ? find_inst<T, 1>(a, k)
                              : kind == 2 ? find_inst<T, 2>(a, k) : find_inst<T, 3>(a, k);
                const BatchInst<T> *in = &a.inst[i];
                const int item = k - (kind == 0 ? in->x_begin : kind == 1 ? in->y_begin
                                      : kind == 2 ? in->c_begin : in->f_begin);
                if (kind == 3)
                    batch_fused<T>(in, item, a.tw, a.lt_shift);
                else
                    batch_pass<T>(kind, in, item, a.tw, a.lt_shift);
            }
            if (!grid_sync(a.ctl, G, a.max_polls)) return;
        }
    }
}

}  // namespace pfc
