// types.hpp -- plain data types shared by the kernels and the host runtime.
#pragma once

#include <stdint.h>

namespace pfc {

// interleaved complex value (re, im)
template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T x, y;
};

// Memory layout of a packed spectrum.  Element (e, row, kx) -- e the index along the last-axis pass
// (z in 3D, y in 2D), row the middle axis (3D y; 0 in 2D), 0 <= kx < M -- lies at
//   row_base(e, row) + col(kx),
//   row_base(e, row) = ((e >> zs) nrows + row) (Mp << zs) + ((e & (Z - 1)) << cs),   Z = 2^zs,
//   col(kx)          = ((kx >> cs) << (zs + cs)) + (kx & (2^cs - 1)):
// rows of pitch Mp >= M, and blocks of Z consecutive planes whose rows are interleaved in chunks of
// 2^cs columns (one 128-byte line), so that the last-axis pass finds Z lines of one column chunk
// next to each other.  zs = 0 is the plain layout of rows of pitch Mp (col(kx) = kx).
struct Pack {
    int64_t nrows, Mp;
    int zs, cs;
    int xnat;  // the x passes visit rows in natural order (see x_row)
    __host__ __device__ int64_t row_base(int64_t e, int64_t row) const
    {
        return (((e >> zs) * nrows + row) * Mp << zs) + ((e & ((int64_t(1) << zs) - 1)) << cs);
    }
    __host__ __device__ int64_t col(int64_t kx) const
    {
        return zs == 0 ? kx : (((kx >> cs) << (zs + cs)) + (kx & ((int64_t(1) << cs) - 1)));
    }
    __host__ __device__ int64_t at(int64_t e, int64_t row, int64_t kx) const { return row_base(e, row) + col(kx); }
    // stride of e, valid for steps of e that are multiples of Z
    __host__ __device__ int64_t e_stride() const { return nrows * Mp; }
    // Row order of the x passes: natural (xnat: position rho is row rho = e nrows + row), or block
    // order, rho = ((e >> zs) nrows + row) Z + (e & (Z - 1)), in which consecutive rows are the Z
    // planes of one block and fill whole runs of lines (measured slower at 2048^3 FP32: its Z rows
    // come from Z planes 16 MiB apart).  Returns the real-field row index e nrows + row of position
    // rho and sets *base to its packed row base.
    __host__ __device__ int64_t x_row(int64_t rho, int64_t *base) const
    {
        if (zs == 0) {
            *base = rho * Mp;
            return rho;
        }
        if (xnat) {  // natural order: position rho is row rho
            const int64_t e = rho / nrows;
            *base = row_base(e, rho - e * nrows);
            return rho;
        }
        const int64_t j = rho & ((int64_t(1) << zs) - 1), q = rho >> zs;
        const int64_t blk = q / nrows, row = q - blk * nrows;
        *base = (q * Mp << zs) + (j << cs);
        return ((blk << zs) + j) * nrows + row;
    }
};

// Addressing of the strided complex FFT (axis_c2c_block): element e = t + k of pencil (batch, col)
// lies at base(batch, col) + elem(t) + k estride, for steps k that are multiples of 2^ezs:
//   base(batch, col) = (batch >> bzs) bstride + ((batch & (2^bzs - 1)) << cs) + column(col),
//   column(col)      = msplit > 0 ? (col / msplit) rstride + pk_col(col % msplit) : pk_col(col),
//   elem(t)          = (t >> ezs) (estride << ezs) + ((t & (2^ezs - 1)) << cs),
// with pk_col the Pack column map of block shift zs.  All shifts zero: base = batch bstride + col,
// elem(t) = t estride.
struct AxisMap {
    int64_t bstride, estride, rstride, msplit;
    int bzs, ezs, zs, cs;
    __host__ __device__ int64_t pk_col(int64_t kx) const
    {
        return zs == 0 ? kx : (((kx >> cs) << (zs + cs)) + (kx & ((int64_t(1) << cs) - 1)));
    }
    __host__ __device__ int64_t base(int64_t batch, int64_t c) const
    {
        const int64_t b = ((batch >> bzs) * bstride) + ((batch & ((int64_t(1) << bzs) - 1)) << cs);
        return b + (msplit > 0 ? (c / msplit) * rstride + pk_col(c % msplit) : pk_col(c));
    }
    __host__ __device__ int64_t elem(int64_t t) const
    {
        return ((t >> ezs) * (estride << ezs)) + ((t & ((int64_t(1) << ezs) - 1)) << cs);
    }
};

// Twiddle buffer layout.  Entries [0, Lt): W_Lt^e = exp(-2 pi i e / Lt) for a power of two Lt.
// After them, per-stage tables: for every stage size N' = Ns R (power of two, 2 <= N' <= Lt) and
// radix R in {2, 4, 8, 16} with R <= N', a block of N' entries whose entry jj R + r is
// W_{N'}^{jj r} (jj < N' / R, r < R).  The R twiddles of one butterfly are adjacent, so a thread
// fetches them with a few wide loads from one address.  The values equal table entries
// W_Lt^{jj r Lt / N'}.
__host__ __device__ constexpr int64_t stage_tw_offset(int64_t Np, int R)
{
    int64_t off = 0;
    for (int64_t n = 2; n < Np; n *= 2)
        for (int r = 2; r <= 16 && r <= n; r *= 2) off += n;
    for (int r = 2; r < R; r *= 2) off += Np;
    return off;
}
// entries after the first Lt that the per-stage tables of every N' <= Lt need
__host__ __device__ constexpr int64_t stage_tw_entries(int64_t Lt) { return stage_tw_offset(2 * Lt, 2); }

// Model parameters in the kernel's precision.  fk[a] = 2 pi / (n_a dx_a): the wavenumber of index
// m on axis a is fk[a] * m (m signed; x indices are 0..M).  Axis 0 is the last-axis pass's axis,
// axis 1 the rows (3D y), axis 2 x.
template <typename T>
struct ModelParams {
    T r, dt, q1sq, R1;
    T fk[3];
    T nl;  // 1: cubic term on; 0: linear PDE only
    int model;
};

// Hydrodynamic PFC spectral updates (kernels.hpp).
// Parameters, in FP64.  fk[0]: last-axis (index e), fk[1]: rows (3D y),
// fk[2]: x wavenumber steps.
struct HydroArgs {
    double fk[3];
    double r, dt, q1sq, R1, nl;
    int model;
    double c;      // dt / rho0
    double gamma;  // viscosity
    double a0;     // width of the Gaussian average
};

// ---- batched persistent form (one entry per instance, in device memory)
template <typename T>
struct BatchInst {
    T *psi;
    cx<T> *state;
    cx<T> *scratch;
    int n0;          // y length (last-axis FFT length)
    int M;           // x length / 2
    int W;           // active pencils per y item
    int tiles;       // y items (M / W)
    int x_items;     // x r2c items
    int c_items;     // x c2r items
    int x_rows, c_rows;  // rows per x r2c / x c2r item
    int f_rows, f_items;  // fused x c2r + x r2c items (between two steps): rows per item, items
    int x_begin, y_begin, c_begin, f_begin;  // first global item of this instance in each pass
    int vx, vy, vc;                 // candidate schedule of the x forward, y and x inverse passes
    T sc;            // 1 / (n0 M)
    ModelParams<T> mp;
};

// Grid-barrier state of the batched kernel.  The arrival counter and the generation the waiters
// poll sit on separate 128-byte lines: on one line, the polling and the arrivals contend for it
// (measured on MI355X, 512 workgroups: 35 us per barrier on one line, 13 us on two).
struct BatchCtl {
    unsigned count;
    unsigned pad0[31];
    unsigned gen;
    int err;
    int pad1[30];
};
static_assert(sizeof(BatchCtl) == 256, "the instance table follows at byte 256");

template <typename T>
struct BatchArgs {
    const BatchInst<T> *inst;  // sorted largest first
    int ninst;
    int x_total, y_total, c_total, f_total;
    const cx<T> *tw;
    int lt_shift;
    BatchCtl *ctl;
    unsigned long long max_polls;
    int64_t nsteps;
};

}  // namespace pfc
