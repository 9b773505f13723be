// launch.hpp -- host-side launchers of the PFC kernels, one set per dtype (float, double).
// Each returns the HIP error of its launch; shapes are validated by the caller (pfc_api.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "types.hpp"

namespace pfc {

// Geometry of a 2D/3D grid as the kernels see it.
struct Geom {
    int ndim;
    int64_t n0, n1, nx;  // 2D: n0 = y, n1 = 1 (unused), nx = x; 3D: z, y, x
    int64_t M;           // nx / 2
    int64_t nrows;       // rows of the last-axis pass: n1 (3D) or 1 (2D)
    int64_t xrows;       // rows of the x pass: n0 * nrows
    int lt_shift;        // log2 of the twiddle table length
    bool nt;             // non-temporal loads/stores of the grids in the step and FFT passes
    // twiddle table of each pass, as an entry offset from the plan's twiddle buffer: 0 (the
    // power-of-two tables) or the own table of a length that is not a power of two
    int64_t tw_x, tw_y, tw_last;
    // layout of the packed spectra (Pack in types.hpp): row pitch (0: M), plane-block and column-chunk
    // shifts; zero is the plain layout
    int64_t Mp = 0;
    int zs = 0, cs = 0;
    int xnat = 0;  // x passes in natural row order
};

// The Pack of a geometry.
inline Pack pack_of(const Geom &g) { return Pack{g.nrows, g.Mp > 0 ? g.Mp : g.M, g.zs, g.cs, g.xnat}; }

// A layout the kernels can address: shifts in range, pitch >= M, and with plane blocks a pitch of
// whole column chunks and a last-axis length of whole blocks.  Every launcher of a packed-layout
// kernel checks it, so a bad geometry is an error, not an out-of-bounds access.
inline bool layout_ok(const Geom &g)
{
    const int64_t Mp = g.Mp > 0 ? g.Mp : g.M;
    if (g.zs < 0 || g.zs > 3 || g.cs < 0 || g.cs > 4 || Mp < g.M) return false;
    if (g.zs == 0) return true;
    return g.ndim == 3 && Mp % (int64_t(1) << g.cs) == 0 && g.n0 % (int64_t(1) << g.zs) == 0;
}

// Lengths other than powers of two that have compiled schedules (factors 2, 3, 5, 7); a grid axis
// of length n needs n here (y and last axis) or n / 2 here (x).
constexpr int kMixedLengths[] = {6, 10, 12, 14, 15, 20, 30, 60, 150, 375, 700, 750, 1400};
inline bool mixed_length(int64_t n)
{
    for (int m : kMixedLengths)
        if (n == m) return true;
    return false;
}

// `variant`: candidate schedule of the pass (0 = default); only the step's passes (x r2c with the
// cube, y forward/inverse, last-axis STEP, x c2r) have more than one candidate.
template <typename T>
hipError_t launch_x_r2c(const Geom &g, const T *in, cx<T> *out, bool cube, const cx<T> *tw, hipStream_t s,
                        int variant = 0);

template <typename T>
hipError_t launch_x_c2r(const Geom &g, const cx<T> *in, T *out, const cx<T> *tw, hipStream_t s, int variant = 0);

// fused x pass between two steps, in place on the packed spectrum: x c2r (1/N), cube, x r2c; on the
// default x schedules, where x_fused_ok says the geometry has it
template <typename T>
hipError_t launch_x_c2r_r2c(const Geom &g, cx<T> *data, const cx<T> *tw, hipStream_t s);
template <typename T>
bool x_fused_ok(const Geom &g);
// whether the last-axis passes can address blocks of 2^zs z planes (their element steps are
// multiples of the block)
template <typename T>
bool z_blocks_ok(const Geom &g, int zs);

// adjoint epilogue: out = mu - c3 psi_n^2 nu; partial[block] = sum nu psi_np1.  Returns the number
// of partials through *nblocks.
template <typename T>
hipError_t launch_x_c2r_adjoint(const Geom &g, const cx<T> *mu, const cx<T> *nu, const T *psi_n, const T *psi_np1,
                                T *out, T c3, double *partial, int64_t *nblocks, const cx<T> *tw, hipStream_t s);

// y-axis (3D middle axis) complex FFT, in place; dir = -1 forward, +1 inverse.
template <typename T>
hipError_t launch_y_c2c(const Geom &g, cx<T> *data, int dir, const cx<T> *tw, hipStream_t s, int variant = 0);

// last-axis complex FFT, forward, out of place, packed in and out (no update).
template <typename T>
hipError_t launch_last_fwd(const Geom &g, const cx<T> *src, cx<T> *dst, const cx<T> *tw, hipStream_t s);

// last-axis complex FFT (dir = -1 forward, +1 inverse), out of place or in place, packed in and out.
template <typename T>
hipError_t launch_last_c2c(const Geom &g, const cx<T> *src, cx<T> *dst, int dir, const cx<T> *tw, hipStream_t s);

// last-axis inverse FFT of the spectral derivative i k of src along a grid role (0 last axis,
// 1 rows, 2 x; wavenumber step fk; k = 0 at a Nyquist index), out of place
template <typename T>
hipError_t launch_last_c2c_deriv(const Geom &g, const cx<T> *src, cx<T> *dst, int role, double fk, const cx<T> *tw,
                                 hipStream_t s);

// x_c2r with the hydrodynamic epilogue: out = w * x (+ out when add), w a real field
template <typename T>
hipError_t launch_x_c2r_mac(const Geom &g, const cx<T> *in, T *out, const T *w, bool add, const cx<T> *tw,
                            hipStream_t s);

// hydrodynamic spectral updates (kernels.hpp), in place: HY_PSI / HY_MU / HY_VEL
template <typename T>
hipError_t launch_spec_update(const Geom &g, int op, cx<T> *out, const cx<T> *x0, const cx<T> *x1,
                              const HydroArgs &h, hipStream_t s);

enum LastMode { LAST_STEP = 0, LAST_R2C_NATURAL = 1, LAST_C2R_NATURAL = 2, LAST_ADJOINT = 3 };
enum HydroOp { HYDRO_PSI = 0, HYDRO_MU = 1, HYDRO_VEL = 2 };  // the spec_update_kernel modes

template <typename T>
hipError_t launch_last(const Geom &g, int mode, const cx<T> *src, cx<T> *dst, cx<T> *dst2, cx<T> *state,
                       const ModelParams<T> &mp, const cx<T> *tw, hipStream_t s, int variant = 0);

// number of candidate schedules of each step pass for this geometry (index as pfc_step_timed's
// passes); used by the autotuner
int step_candidates(const Geom &g, int pass);

// reductions; every launcher uses exactly kReduceBlocks partials
constexpr int kReduceBlocks = 1024;
template <typename T>
hipError_t launch_set_mass(const T *psi, int64_t n, double *partial, cx<T> *state, hipStream_t s);
template <typename T>
hipError_t launch_energy(const Geom &g, const T *psi, const cx<T> *state, const double fk[3], double r, double q1sq,
                         double R1, int model, double dV, double *partial, double *out, hipStream_t s);
template <typename T>
hipError_t launch_export(const Geom &g, const cx<T> *state, cx<T> *out, hipStream_t s);
hipError_t launch_accumulate(const double *partial, int np, double coef, double *acc, hipStream_t s);

// batched persistent kernel: kBatchThreads threads per workgroup, `grid` workgroups (all resident)
template <typename T>
hipError_t launch_batch(const BatchArgs<T> &a, int grid, hipStream_t s);
template <typename T>
hipError_t batch_blocks_per_cu(int *blocks);
constexpr int kBatchThreadsHost = 512;
constexpr int kBatchMaxInstHost = 256;
// rows per x-forward / x-inverse item and pencils per y item of the batched kernel for an n0 x 2M
// instance of dtype FP64 (f64) or FP32 with candidate schedules (vx, vy, vc) (returns false for
// unsupported lengths/candidates)
bool batch_tiles(int n0, int M, int vx, int vy, int vc, bool f64, int *x_rows, int *c_rows, int *y_pencils);
// number of candidates of batched pass `pass` (0 x forward, 1 y, 2 x inverse) for an n0 x 2M instance
int batch_candidates(int n0, int M, int pass);

}  // namespace pfc
