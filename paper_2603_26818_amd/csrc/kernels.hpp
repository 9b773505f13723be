// kernels.hpp -- HIP kernels of the PFC hot path (gfx950).
//
// Layouts (C-order, x fastest; M = n_x / 2):
//   real field      [rows][2M]                      rows = n0 n1 (3D) or n0 (2D)
//   packed spectrum [n0][nrows][M] complex           nrows = n1 (3D) or 1 (2D)
//     column kx in 1..M-1 holds X(kx); column 0 holds X(0) + i X(M): the planes kx = 0 and
//     kx = n_x/2 are spectra of real data and share one complex plane.  After the transforms along
//     the other axes, column 0 holds Z = X0_hat + i XN_hat, and the two Hermitian planes are
//         X0_hat(k) = (Z(k) + conj Z(-k)) / 2,   XN_hat(k) = -i (Z(k) - conj Z(-k)) / 2.
//   natural half    [n0][nrows][M+1] complex
//
// Pass schedule of one step (arxiv 2603.26818, Listing 1: cube, forward transform, update of the
// spectrum, inverse transform), 3D:
//   x_r2c (cube prologue) -> y forward -> last-axis (z forward, update, z inverse) -> y inverse
//   -> x_c2r (1/N epilogue);   2D: x_r2c -> last-axis along y -> x_c2r.
#pragma once

#include "fft_core.hpp"

namespace pfc {

// ------------------------------------------------------------------------------------------------
// L(q) and the implicit multiplier, in the kernel's precision (ModelParams in types.hpp).
template <typename T>
__device__ __forceinline__ T corr_op(const ModelParams<T> &m, T q)
{
    T a = (T(1) - q) * (T(1) - q);
    if (m.model == 0) return a;
    T b = m.q1sq - q;
    return a * (b * b + m.R1);
}

// A(q) = 1 / (1 + dt q (r + L(q))); exactly 1 at q = 0.  FP32 takes the hardware reciprocal
// (within 1 ulp, exact for 1); FP64 divides.
template <typename T>
__device__ __forceinline__ T amult(const ModelParams<T> &m, T q)
{
    const T d = T(1) + m.dt * q * (m.r + corr_op(m, q));
    if constexpr (sizeof(T) == 4)
        return __builtin_amdgcn_rcpf(d);
    else
        return T(1) / d;
}

// Loads and stores of the streamed grids.  NT marks them non-temporal: on grids far larger than
// the caches, nothing a pass touches is read again before it is evicted.
template <bool NT, typename T>
__device__ __forceinline__ cx<T> ld_grid(const cx<T> *p)
{
    if constexpr (NT) {
        typedef T v2 __attribute__((ext_vector_type(2)));
        const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2 *>(p));
        return {v.x, v.y};
    } else {
        return *p;
    }
}
template <bool NT, typename T>
__device__ __forceinline__ void st_grid(cx<T> *p, cx<T> a)
{
    if constexpr (NT) {
        typedef T v2 __attribute__((ext_vector_type(2)));
        v2 v;
        v.x = a.x;
        v.y = a.y;
        __builtin_nontemporal_store(v, reinterpret_cast<v2 *>(p));
    } else {
        *p = a;
    }
}

__device__ __forceinline__ int signed_index(int64_t i, int64_t n) { return (int)(i <= n / 2 ? i : i - n); }

// (-e) mod L for 0 <= e < L
template <int L>
__device__ __forceinline__ int neg_mod(int e)
{
    if constexpr (is_pow2c(L))
        return (L - e) & (L - 1);
    else
        return e == 0 ? 0 : L - e;
}

// x-pass split twiddle W_{2M}^k, 0 <= k < M: from the W_Lt table, or from the length's own table
// (lengths that are not powers of two; layout in fft_core.hpp)
template <typename T, int M>
__device__ __forceinline__ cx<T> split_twiddle(const cx<T> *__restrict__ tw, int lt_shift, int k)
{
    if constexpr (is_pow2c(M))
        return tw[k << (lt_shift - ilog2c(2 * M))];
    else
        return tw[MixTable<M>::split + k];
}

// ------------------------------------------------------------------------------------------------
// Block-wide FP64 sum; the result is valid in thread 0.  red: >= blockDim.x/64 doubles of LDS.
__device__ __forceinline__ double block_sum(double v, double *red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x + 63) / 64; ++i) s += red[i];
    return s;
}

// ------------------------------------------------------------------------------------------------
// x axis, forward: one row of 2M reals -> M packed complex values.
// z[m] = x[2m] + i x[2m+1] (cubed first when CUBE), Z = FFT_M(z), then for k = 1..M-1
//   X(k) = E + W_{2M}^k O,  E = (Z(k) + conj Z(M-k)) / 2,  O = -i (Z(k) - conj Z(M-k)) / 2,
// and slot 0 = (Re Z0 + Im Z0) + i (Re Z0 - Im Z0) = X(0) + i X(M).
// rows per workgroup of the x pass: about 256 threads
template <class PL>
struct XRows {
    static constexpr int value = (256 / PL::Tp) > 64 ? 64 : ((256 / PL::Tp) < 1 ? 1 : 256 / PL::Tp);
};

// Padded LDS rows of the x pass (PAD, power-of-two rows of M complex values): 16 spare bytes after
// every 256 bytes of a row, i.e. after every S = 256 / sizeof(cx<T>) elements (M, if shorter).  With
// 64 banks of 4 bytes, a Stockham stage write puts neighbouring threads R elements apart; unpadded,
// the threads of a power-of-two row then meet on a few bank positions of each 256-byte sweep (up to
// 16 ways for the first stage of a 512-point r2c).  The 16-byte step keeps 16-byte alignment and
// fixed offsets between one thread's elements, so merged and paired LDS accesses stay possible.
template <typename T, int M>
struct XPad {
    static constexpr int S0 = 256 / (int)sizeof(cx<T>);
    static constexpr int S = S0 < M ? S0 : M;
    static constexpr int k = 16 / (int)sizeof(cx<T>);
    static constexpr int shift = ilog2c(S);
};
template <typename T, int M, bool PAD>
struct XPitch {
    static_assert(!PAD || is_pow2c(M), "padded rows are powers of two");
    static constexpr int value = PAD ? M + XPad<T, M>::k * (M / XPad<T, M>::S) : M;
};
template <typename T, int M, bool PAD>
__device__ __forceinline__ int xidx(int e)
{
    if constexpr (PAD)
        return e + XPad<T, M>::k * (e >> XPad<T, M>::shift);
    else
        return e;
}

// Identity layout of a packed spectrum with rows of M values (2D plans, the batched form).
__host__ __device__ inline Pack row_pack(int64_t M) { return Pack{1, M, 0, 0}; }

// One block of ROWS rows (block index `bid`); `sh` holds ROWS * XPitch<T, M, PAD> LDS slots.
// Uses threads 0 .. ROWS*Tp-1, which must be all threads of the workgroup.  FROM_LDS: the rows'
// reals are not read from `in` but from `sh` (row p at sh[p LD], LD the row pitch, as packed
// pairs, contiguous), where the caller
// has left them.  Output row rr (= e nrows + row) goes to the layout `pk`.
template <typename T, class PL, int ROWS, bool CUBE, bool PAD = false, bool NT = false, bool FROM_LDS = false>
__device__ __forceinline__ void x_r2c_block(const T *__restrict__ in, cx<T> *__restrict__ out, int64_t nrows,
                                            const cx<T> *__restrict__ tw, int lt_shift, int64_t bid, cx<T> *sh,
                                            const Pack &pk)
{
    constexpr int M = PL::L, Tp = PL::Tp, R0 = PL::first, Rl = PL::last, Rmax = PL::Rmax;
    constexpr int LD = XPitch<T, M, PAD>::value;  // row pitch in LDS
    const int tid = threadIdx.x, p = tid / Tp, t = tid - p * Tp;
    const int64_t rho = bid * ROWS + p;  // position in the pass's row order (Pack::x_row)
    const bool valid = rho < nrows;
    int64_t obase;
    const int64_t row = pk.x_row(valid ? rho : 0, &obase);
    const cx<T> *src = FROM_LDS ? sh + p * LD : reinterpret_cast<const cx<T> *>(in) + row * M;
    cx<T> v[Rmax];
#pragma unroll
    for (int b = 0; b < PL::nb(R0); ++b)
        if (PL::jok(t + b * Tp, R0))
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            cx<T> z;
            if constexpr (FROM_LDS)
                z = src[t + b * Tp + r * (M / R0)];
            else
                z = valid ? ld_grid<NT>(&src[t + b * Tp + r * (M / R0)]) : cx<T>{T(0), T(0)};
            if constexpr (CUBE) z = {z.x * z.x * z.x, z.y * z.y * z.y};
            v[b * R0 + r] = z;
        }
    auto lds = [&](int e) -> cx<T> & { return sh[p * LD + xidx<T, M, PAD>(e)]; };
    fft_stages<T, PL, -1, TW_LT>(v, t, lds, tw, lt_shift);  // measured faster here than TW_STAGE
    __syncthreads();
#pragma unroll
    for (int b = 0; b < PL::nb(Rl); ++b)
        if (PL::jok(t + b * Tp, Rl))
#pragma unroll
        for (int r = 0; r < Rl; ++r) lds(t + b * Tp + r * (M / Rl)) = v[b * Rl + r];
    __syncthreads();
    cx<T> *dst = out + obase;
    const T h = T(0.5);
#pragma unroll
    for (int b = 0; b < PL::nb(Rl); ++b)
        if (PL::jok(t + b * Tp, Rl))
#pragma unroll
        for (int r = 0; r < Rl; ++r) {
            const int k = t + b * Tp + r * (M / Rl);
            const cx<T> Zk = v[b * Rl + r];
            cx<T> X;
            if (k == 0) {
                X = {Zk.x + Zk.y, Zk.x - Zk.y};
            } else {
                const cx<T> Zp = lds(M - k);
                const cx<T> E = {(Zk.x + Zp.x) * h, (Zk.y - Zp.y) * h};
                const cx<T> O = {(Zk.y + Zp.y) * h, (Zp.x - Zk.x) * h};
                X = E + cmul(split_twiddle<T, M>(tw, lt_shift, k), O);
            }
            if (valid) st_grid<NT>(&dst[pk.col(k)], X);
        }
}

template <typename T, class PL, int ROWS, bool CUBE, bool PAD = false, bool NT = false>
__global__ __launch_bounds__(ROWS *PL::Tp) void x_r2c_kernel(const T *__restrict__ in, cx<T> *__restrict__ out,
                                                              int64_t nrows, const cx<T> *__restrict__ tw,
                                                              int lt_shift, Pack pk)
{
    __shared__ cx<T> sh[ROWS * XPitch<T, PL::L, PAD>::value];
    x_r2c_block<T, PL, ROWS, CUBE, PAD, NT>(in, out, nrows, tw, lt_shift, blockIdx.x, sh, pk);
}

// ------------------------------------------------------------------------------------------------
// x axis, inverse: M packed complex -> 2M reals (times `scale`).  For k = 1..M-1
//   E = (X(k) + conj X(M-k)) / 2,  O = conj(W_{2M}^k) (X(k) - conj X(M-k)) / 2,  Z(k) = E + i O,
// Z(0) = ((X0 + XM) + i (X0 - XM)) / 2 from the packed slot; z = IFFT_M(Z) (unnormalised);
// x[2m] = Re z[m] * scale, x[2m+1] = Im z[m] * scale.
//
// EPI_PLAIN stores x.  EPI_ADJOINT transforms two spectra (mu from `in`, in the layout `pk`; nu
// from `in2`, always in the plain layout of rows of M, so that nu's row r covers the same bytes as
// the real row r) and stores
//   out = mu - c3 * psi_n^2 * nu,   and writes the block's FP64 sum of nu * psi_np1 to partial[].
// `in2` and `out` may be the same buffer: each block reads its rows completely before writing them.
// EPI_MAC (hydrodynamic step) stores out = w * x (+ out when `add`), w a real field.
enum { EPI_PLAIN = 0, EPI_ADJOINT = 1, EPI_MAC = 2 };

template <typename T>
struct AdjEpi {
    const cx<T> *in2;
    const T *psi_n;
    const T *psi_np1;
    T c3;
    double *partial;
    const T *w;  // EPI_MAC
    int add;     // EPI_MAC
};

// Pre-combination of one row for the c2r: own elements X(k) from `src` (column k at src[pk.col(k)]);
// the mirror X(M-k) either through LDS (PG = false) or straight from `src` (PG = true: a second,
// reversed but coalesced load of the same cache lines, without the LDS round trip and its barrier).
template <typename T, class PL, int ROWS, bool PAD, bool PG = false, bool NT = false>
__device__ __forceinline__ void x_c2r_row(cx<T> *v, const cx<T> *src, bool valid, int t, cx<T> *rowlds,
                                          const cx<T> *__restrict__ tw, int lt_shift, const Pack &pk)
{
    constexpr int M = PL::L, Tp = PL::Tp, R0 = PL::first, Rmax = PL::Rmax;
    cx<T> mir[PG ? Rmax : 1];
    if constexpr (PG) {
#pragma unroll
        for (int b = 0; b < PL::nb(R0); ++b)
            if (PL::jok(t + b * Tp, R0))
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                const int k = t + b * Tp + r * (M / R0);
                v[b * R0 + r] = valid ? ld_grid<NT>(&src[pk.col(k)]) : cx<T>{T(0), T(0)};
                mir[b * R0 + r] = valid ? ld_grid<NT>(&src[pk.col(neg_mod<M>(k))]) : cx<T>{T(0), T(0)};
            }
    } else {
        __syncthreads();
#pragma unroll
        for (int b = 0; b < PL::nb(R0); ++b)
            if (PL::jok(t + b * Tp, R0))
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                const int k = t + b * Tp + r * (M / R0);
                v[b * R0 + r] = valid ? ld_grid<NT>(&src[pk.col(k)]) : cx<T>{T(0), T(0)};
                rowlds[xidx<T, M, PAD>(k)] = v[b * R0 + r];
            }
        __syncthreads();
    }
    const T h = T(0.5);
#pragma unroll
    for (int b = 0; b < PL::nb(R0); ++b)
        if (PL::jok(t + b * Tp, R0))
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int k = t + b * Tp + r * (M / R0);
            const cx<T> a = v[b * R0 + r];
            if (k == 0) {
                v[b * R0 + r] = {(a.x + a.y) * h, (a.x - a.y) * h};
            } else {
                cx<T> c;  // X(M-k); conj taken below
                if constexpr (PG)
                    c = mir[b * R0 + r];
                else
                    c = rowlds[xidx<T, M, PAD>(M - k)];
                const cx<T> E = {(a.x + c.x) * h, (a.y - c.y) * h};
                const cx<T> D = {(a.x - c.x) * h, (a.y + c.y) * h};
                const cx<T> O = cmul(conj(split_twiddle<T, M>(tw, lt_shift, k)), D);
                v[b * R0 + r] = {E.x - O.y, E.y + O.x};
            }
        }
}

// TO_LDS (EPI_PLAIN): the scaled reals of row p are left in sh[p LD] (LD the row pitch, as packed
// pairs, contiguous) instead of being stored to `out`.
template <typename T, class PL, int ROWS, int EPI, bool PAD = false, bool PG = false, bool NT = false,
          bool TO_LDS = false>
__device__ __forceinline__ void x_c2r_block(const cx<T> *in, T *out, int64_t nrows, const cx<T> *__restrict__ tw,
                                            int lt_shift, T sc, const AdjEpi<T> &ea, int64_t bid, cx<T> *sh,
                                            const Pack &pk)
{
    static_assert(!TO_LDS || EPI == EPI_PLAIN, "staging only for the plain epilogue");
    constexpr int M = PL::L, Tp = PL::Tp, Rl = PL::last, Rmax = PL::Rmax;
    constexpr int LD = XPitch<T, M, PAD>::value;
    const int tid = threadIdx.x, p = tid / Tp, t = tid - p * Tp;
    const int64_t rho = bid * ROWS + p;  // position in the pass's row order (Pack::x_row)
    const bool valid = rho < nrows;
    int64_t ibase;
    const int64_t r0 = pk.x_row(valid ? rho : 0, &ibase);  // real-field row
    auto lds = [&](int e) -> cx<T> & { return sh[p * LD + xidx<T, M, PAD>(e)]; };
    cx<T> v[Rmax];
    x_c2r_row<T, PL, ROWS, PAD, PG, NT>(v, in + ibase, valid, t, &sh[p * LD], tw, lt_shift, pk);
    fft_stages<T, PL, +1>(v, t, lds, tw, lt_shift);
    cx<T> *dst = reinterpret_cast<cx<T> *>(out) + r0 * M;
    if constexpr (EPI == EPI_MAC) {
        if (valid) {
            const cx<T> *wr = reinterpret_cast<const cx<T> *>(ea.w) + r0 * M;
#pragma unroll
            for (int b = 0; b < PL::nb(Rl); ++b)
                if (PL::jok(t + b * Tp, Rl))
#pragma unroll
                    for (int r = 0; r < Rl; ++r) {
                        const int m = t + b * Tp + r * (M / Rl);
                        const cx<T> x = scale(v[b * Rl + r], sc), w = wr[m];
                        cx<T> o = {w.x * x.x, w.y * x.y};
                        if (ea.add) o = o + dst[m];
                        dst[m] = o;
                    }
        }
    } else if constexpr (EPI == EPI_PLAIN && TO_LDS) {
        __syncthreads();  // every thread of the row is past its last exchange read
#pragma unroll
        for (int b = 0; b < PL::nb(Rl); ++b)
            if (PL::jok(t + b * Tp, Rl))
#pragma unroll
            for (int r = 0; r < Rl; ++r) sh[p * LD + t + b * Tp + r * (M / Rl)] = scale(v[b * Rl + r], sc);
    } else if constexpr (EPI == EPI_PLAIN) {
        if (valid) {
#pragma unroll
            for (int b = 0; b < PL::nb(Rl); ++b)
                if (PL::jok(t + b * Tp, Rl))
#pragma unroll
                for (int r = 0; r < Rl; ++r)
                    st_grid<NT>(&dst[t + b * Tp + r * (M / Rl)], scale(v[b * Rl + r], sc));
        }
    } else {
        cx<T> w[Rmax];
        x_c2r_row<T, PL, ROWS, PAD, PG>(w, ea.in2 + r0 * M, valid, t, &sh[p * LD], tw, lt_shift, row_pack(M));
        fft_stages<T, PL, +1>(w, t, lds, tw, lt_shift);
        const cx<T> *pn = reinterpret_cast<const cx<T> *>(ea.psi_n) + r0 * M;
        const cx<T> *pn1 = reinterpret_cast<const cx<T> *>(ea.psi_np1) + r0 * M;
        double acc = 0.0;
        if (valid) {
#pragma unroll
            for (int b = 0; b < PL::nb(Rl); ++b)
                if (PL::jok(t + b * Tp, Rl))
#pragma unroll
                for (int r = 0; r < Rl; ++r) {
                    const int m = t + b * Tp + r * (M / Rl);
                    const cx<T> mu = scale(v[b * Rl + r], sc), nu = scale(w[b * Rl + r], sc);
                    const cx<T> a = pn[m], c = pn1[m];
                    dst[m] = {mu.x - ea.c3 * a.x * a.x * nu.x, mu.y - ea.c3 * a.y * a.y * nu.y};
                    acc += (double)nu.x * (double)c.x + (double)nu.y * (double)c.y;
                }
        }
        __shared__ double red[16];
        const double s = block_sum(acc, red);
        if (threadIdx.x == 0) ea.partial[bid] = s;
    }
}

template <typename T, class PL, int ROWS, int EPI, bool PAD = false, bool PG = false, bool NT = false>
__global__ __launch_bounds__(ROWS *PL::Tp) void x_c2r_kernel(const cx<T> *in, T *out, int64_t nrows,
                                                              const cx<T> *__restrict__ tw, int lt_shift, T sc,
                                                              AdjEpi<T> ea, Pack pk)
{
    __shared__ cx<T> sh[ROWS * XPitch<T, PL::L, PAD>::value];
    x_c2r_block<T, PL, ROWS, EPI, PAD, PG, NT>(in, out, nrows, tw, lt_shift, sc, ea, blockIdx.x, sh, pk);
}

// ------------------------------------------------------------------------------------------------
// Pencils per workgroup of the strided passes: 128-byte rows (16 FP32 / 8 FP64 complex) as long as
// the workgroup's LDS tile stays within 128 KB.
// x pass between two steps (batched runs, and the single-plan step within one call): the inverse x
// transform of one step (x c2r) and the forward x transform with the cube of the next (x r2c), over
// the same rows, with the field between them kept in LDS: a workgroup takes R rows, runs the c2r
// schedule PLI on them in groups of RI rows (each group leaving its reals in its rows' LDS slots),
// then the r2c schedule PLF in groups of RF rows reading those slots.  The field of the intermediate
// step is never stored.  Arithmetic identical to x_c2r_kernel followed by x_r2c_kernel with the
// cube.  The single-plan step runs it with one wavefront per workgroup (at 512^3: 4 rows in padded
// LDS rows, 8.5 KB, many workgroups per CU), which keeps the row FFTs, that bound it at half the
// memory traffic, overlapped; 256-thread workgroups measured no faster than the two separate passes.
template <class PLI, class PLF, int NTH = 256>
struct XFused {
    static constexpr int RI = NTH / PLI::Tp < 1 ? 1 : NTH / PLI::Tp;
    static constexpr int RF = NTH / PLF::Tp < 1 ? 1 : NTH / PLF::Tp;
    static constexpr int R = RI > RF ? RI : RF;
    static constexpr int threads = RI * PLI::Tp;
    // both schedules fill the same workgroup, and a group of either kind tiles the R rows
    static constexpr bool ok = RI * PLI::Tp == RF * PLF::Tp && R % RI == 0 && R % RF == 0;
};
// One block of R rows (block index `bid`) of packed spectra in the layout `pk`; `sh` holds
// R XPitch<T, M, PAD> LDS slots; NTH threads.  In place (in == out) is safe: the block reads all its
// rows before it writes.
template <typename T, class PLI, class PLF, int NTH, bool NT = false, bool PAD = false>
__device__ __forceinline__ void x_c2r_r2c_block(const cx<T> *in, cx<T> *out, int64_t nrows,
                                                const cx<T> *__restrict__ tw, int lt_shift, T sc, int64_t bid,
                                                cx<T> *sh, const Pack &pk)
{
    using F = XFused<PLI, PLF, NTH>;
    static_assert(F::ok && PLI::L == PLF::L, "schedules must share the workgroup");
    constexpr int LD = XPitch<T, PLI::L, PAD>::value;
    const AdjEpi<T> ea{};
#pragma unroll
    for (int s = 0; s < F::R / F::RI; ++s)
        x_c2r_block<T, PLI, F::RI, EPI_PLAIN, PAD, false, NT, true>(in, nullptr, nrows, tw, lt_shift, sc, ea,
                                                                    bid * (F::R / F::RI) + s, sh + s * F::RI * LD,
                                                                    pk);
    __syncthreads();  // all staged rows written
#pragma unroll
    for (int s = 0; s < F::R / F::RF; ++s)
        x_r2c_block<T, PLF, F::RF, true, PAD, NT, true>(nullptr, out, nrows, tw, lt_shift, bid * (F::R / F::RF) + s,
                                                        sh + s * F::RF * LD, pk);
}

// The fused x pass of the single-plan step between two steps: one workgroup of NTH threads (one
// wavefront in the step) takes XFused<PLI, PLF, NTH>::R rows of the packed spectrum, in place.
template <typename T, class PLI, class PLF, int NTH, bool NT, bool PAD>
__global__ __launch_bounds__(NTH) void x_c2r_r2c_kernel(cx<T> *data, int64_t nrows, const cx<T> *__restrict__ tw,
                                                        int lt_shift, T sc, Pack pk)
{
    __shared__ cx<T> sh[XFused<PLI, PLF, NTH>::R * XPitch<T, PLI::L, PAD>::value];
    x_c2r_r2c_block<T, PLI, PLF, NTH, NT, PAD>(data, data, nrows, tw, lt_shift, sc, blockIdx.x, sh, pk);
}


template <typename T, int L>
struct WMax {
    static constexpr int pref = 128 / (int)sizeof(cx<T>);
    static constexpr int cap = (131072 / (L * (int)sizeof(cx<T>))) < 2 ? 2 : (131072 / (L * (int)sizeof(cx<T>)));
    static constexpr int value = pref < cap ? pref : cap;
};

// Tile of the strided passes (y, and the last-axis step) per length: W pencils per workgroup,
// E elements per thread (0: the schedule's largest radix), G LDS groups (fft_stages), state
// prefetch in the step.  Default: WMax pencils, one LDS area.  Long FP32 pencils, measured on
// MI355X: at 1024, 16 pencils with 32 elements per thread and two LDS groups (512 threads, 64 KB:
// two workgroups per CU); at 2048 the same with 1024 threads and 128 KB, which keeps the column
// tile a whole 128-byte line (the default 8 pencils leave 64-byte tiles: y 19.1 -> 15.9 ms and
// z 63 -> 50 ms at 2048^3).
template <typename T, int L>
struct PencilTile {
    static constexpr int W = WMax<T, L>::value, E = 0, G = 1;
    static constexpr bool PF = is_pow2c(L);  // mixed radices hold up to 30 elements per thread
};
template <>
struct PencilTile<float, 1024> {
    static constexpr int W = 16, E = 32, G = 2;
    static constexpr bool PF = false;
};
template <>
struct PencilTile<float, 1400> {  // 16 pencils of 1400 (800 threads) in two LDS groups (88 KB)
    static constexpr int W = 16, E = 0, G = 2;
    static constexpr bool PF = false;
};
template <>
struct PencilTile<double, 1400> {  // 8 pencils (128-byte tiles) in two LDS groups (88 KB)
    static constexpr int W = 8, E = 0, G = 2;
    static constexpr bool PF = false;
};
template <>
struct PencilTile<float, 2048> {
    static constexpr int W = 16, E = 32, G = 2;  // whole 128-byte lines; 1024 threads, 128 KB
    static constexpr bool PF = false;
};
template <class PL, int E>
using SpreadIf = std::conditional_t<(E > 0), Spread<PL, (E > 0 ? E : PL::Rmax)>, PL>;

// The tile and the radix schedule of a strided-pass candidate C: a plain schedule takes its
// length's PencilTile; a Tiled candidate (fft_core.hpp) its own, W = SEGB / sizeof(complex).
template <typename T, class C, class = void>
struct TileOf {
    using tile = PencilTile<T, C::L>;
    using plan = C;
};
template <typename T, class C>
struct TileOf<T, C, std::void_t<typename C::plan>> {
    struct tile {
        static constexpr int W = C::seg_bytes / (int)sizeof(cx<T>), E = C::elems, G = C::groups;
        static constexpr bool PF = C::prefetch;
    };
    using plan = typename C::plan;
};

// ------------------------------------------------------------------------------------------------
// Workgroup order for column tiles narrower than a 128-byte line.  Consecutive workgroups are
// dispatched to the 8 XCDs in turn, so workgroups b, b + 8, ..., b + 8 (G - 1) share one XCD and
// its L2; they are given G adjacent tiles, which then share every line in that L2 instead of
// fetching and writing it from G XCDs.  A permutation of [0, n): an incomplete last group keeps
// its indices.
__device__ __forceinline__ int64_t xcd_tile_order(int64_t b, int64_t n, int G)
{
    if (G <= 1) return b;
    const int64_t span = 8 * (int64_t)G, full = n - n % span;
    if (b >= full) return b;
    const int64_t grp = b / span, w = b - grp * span;
    return (grp * 8 + (w & 7)) * G + (w >> 3);
}

// Spectral first derivative applied on load by the strided FFT (DERIV): multiplies element e of
// pencil column col = row * M + kx by i k, k along `role` (0: this axis, index e of length L; 1: the
// rows; 2: x), with k = 0 at a Nyquist index (a first derivative of a real field has no real Nyquist
// component), computed in FP64 and rounded once.  On the folded column kx = 0 of the packed layout
// the multiplier is the same for both planes (0 for x), so it applies to X0 + i XN as stored.
struct DerivArgs {
    int role;
    double fk;
    int64_t nrows, M;
};

// ------------------------------------------------------------------------------------------------
// Strided complex FFT along one axis, out of place or in place (src == dst).
// Pencil (batch, col), col < ncols, has element e = t + k at am.base(batch, col) + am.elem(t) +
// k am.estride (AxisMap in types.hpp; every step k the schedule takes is a multiple of 2^am.ezs, which
// the launcher checks).  A workgroup handles W adjacent columns (W <= WMAX); its threads are laid out
// column-fastest so each load/store instruction moves W * sizeof(cx) contiguous bytes per element
// row (within one 128-byte column chunk).  `bid` is the logical tile index (see xcd_tile_order).
template <typename T, class PL, int WMAX, int DIR, bool NT = false, int G = 1, bool DERIV = false>
__device__ __forceinline__ void axis_c2c_block(const cx<T> *src, cx<T> *dst, int W, int64_t ncols, const AxisMap &am,
                                               int64_t tiles_per_batch, const cx<T> *__restrict__ tw, int lt_shift,
                                               int64_t bid, cx<T> *sh, const DerivArgs &da = DerivArgs{})
{
    constexpr int L = PL::L, Tp = PL::Tp, R0 = PL::first, Rl = PL::last, Rmax = PL::Rmax;
    const int tid = threadIdx.x, p = tid % WMAX, t = tid / WMAX;
    const int64_t batch = bid / tiles_per_batch, tile = bid - batch * tiles_per_batch;
    const int64_t col = tile * W + p;
    const bool valid = p < W && col < ncols;
    const int64_t base = am.base(batch, valid ? col : 0) + am.elem(t);
    const int64_t estride = am.estride;
    cx<T> v[Rmax];
#pragma unroll
    for (int b = 0; b < PL::nb(R0); ++b)
        if (PL::jok(t + b * Tp, R0))
#pragma unroll
        for (int r = 0; r < R0; ++r)
            v[b * R0 + r] = valid ? ld_grid<NT>(&src[base + (int64_t)(b * Tp + r * (L / R0)) * estride])
                                  : cx<T>{T(0), T(0)};
    if constexpr (DERIV) {
        const int64_t crow = valid ? col / da.M : 0, ckx = valid ? col - crow * da.M : 0;
#pragma unroll
        for (int b = 0; b < PL::nb(R0); ++b)
            if (PL::jok(t + b * Tp, R0))
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                const int e = t + b * Tp + r * (L / R0);
                double k;
                if (da.role == 0)
                    k = (2 * e == L) ? 0.0 : da.fk * signed_index(e, L);
                else if (da.role == 1)
                    k = (2 * crow == da.nrows) ? 0.0 : da.fk * signed_index(crow, da.nrows);
                else
                    k = da.fk * (double)ckx;
                const cx<T> z = v[b * R0 + r];
                v[b * R0 + r] = {(T)(-k * (double)z.y), (T)(k * (double)z.x)};
            }
    }
    constexpr int GW = WMAX / G;  // pencils per LDS group (see fft_stages)
    auto lds = [&](int e) -> cx<T> & { return sh[e * GW + p % GW]; };
    fft_stages<T, PL, DIR, TW_STAGE, G>(v, t, lds, tw, lt_shift, p / GW);
    if (valid) {
#pragma unroll
        for (int b = 0; b < PL::nb(Rl); ++b)
            if (PL::jok(t + b * Tp, Rl))
#pragma unroll
            for (int r = 0; r < Rl; ++r)
                st_grid<NT>(&dst[base + (int64_t)(b * Tp + r * (L / Rl)) * estride], v[b * Rl + r]);
    }
}

// Workgroup order: xg >= 1 as xcd_tile_order; xg == 0: workgroup b (on XCD b mod 8) takes the
// batches congruent to b mod 8, their tiles in order, so each XCD works through whole planes (the
// batches past the last multiple of 8 keep the tile order).  Measured for the y pass at 512^3 FP32:
// 188-192 against 206-219 us; at 750^3 (rows not line-aligned, so neighbouring tiles share lines,
// which now meet in one L2) 1.26 against 1.87 ms; slower for the grouped 2048-point tiles.
__device__ __forceinline__ int64_t plane_xcd_order(int64_t b, int64_t tiles_per_batch, int64_t nblocks)
{
    const int64_t batches = nblocks / tiles_per_batch;
    if (b >= (batches - batches % 8) * tiles_per_batch) return b;
    const int64_t k = b >> 3;
    return ((k / tiles_per_batch) * 8 + (b & 7)) * tiles_per_batch + k % tiles_per_batch;
}

// With batch blocks (am.bzs > 0: 2^bzs batches share the rows of one block), the plane order runs
// over whole blocks, and inside a block over tiles first, then the batches of the block, so that
// consecutive workgroups of an XCD read neighbouring 128-byte chunks.
template <typename T, class PL, int WMAX, int DIR, int OCC = 1, bool NT = false, int G = 1>
__global__ __launch_bounds__(WMAX *PL::Tp, OCC) void axis_c2c_kernel(const cx<T> *src, cx<T> *dst, int W,
                                                                 int64_t ncols, AxisMap am, int64_t tiles_per_batch,
                                                                 const cx<T> *__restrict__ tw, int lt_shift, int xg)
{
    static_assert(WMAX % G == 0, "groups of whole pencils");
    __shared__ cx<T> sh[PL::L * WMAX / G];
    int64_t bid;
    if (xg == 0) {
        const int64_t tb = tiles_per_batch << am.bzs;
        const int64_t u = plane_xcd_order(blockIdx.x, tb, gridDim.x);
        const int64_t sb = u / tb, w = u - sb * tb;
        const int64_t batch = (sb << am.bzs) + (w & ((int64_t(1) << am.bzs) - 1));
        bid = batch * tiles_per_batch + (w >> am.bzs);
    } else {
        bid = xcd_tile_order(blockIdx.x, gridDim.x, xg);
    }
    axis_c2c_block<T, PL, WMAX, DIR, NT, G>(src, dst, W, ncols, am, tiles_per_batch, tw, lt_shift, bid, sh);
}

// Inverse strided FFT of the spectral derivative i k_role of `src` (DerivArgs), out of place.
template <typename T, class PL, int WMAX>
__global__ __launch_bounds__(WMAX *PL::Tp) void axis_c2c_deriv_kernel(const cx<T> *src, cx<T> *dst, int W,
                                                                   int64_t ncols, AxisMap am,
                                                                   const cx<T> *__restrict__ tw, int lt_shift,
                                                                   DerivArgs da)
{
    __shared__ cx<T> sh[PL::L * WMAX];
    axis_c2c_block<T, PL, WMAX, +1, false, 1, true>(src, dst, W, ncols, am, (ncols + W - 1) / W, tw, lt_shift,
                                                    blockIdx.x, sh, da);
}

// ------------------------------------------------------------------------------------------------
// Last-axis pass (z in 3D, y in 2D): FFT length L = n0 along the slowest axis, rows = n1 (3D) or 1
// (2D), M columns per row.  Element e of pencil (row, kx) sits at e*nrows*M + row*M + kx.
//
// Column kx = 0 pencils need their mirror pencil (row' = -row mod nrows, element -e mod L) to
// separate the two folded planes.  Tiles: W adjacent columns of one row for column tiles >= 1;
// column tile 0 is covered by "pair tiles" that take W/2 columns of row a and the same W/2 columns
// of its mirror row b (pairs (0, nrows/2) and (i, nrows-i)), so a pencil and its mirror always
// share a workgroup.  With nrows == 1 every kx = 0 pencil is its own mirror.
enum { LA_STEP = 0, LA_R2C_NATURAL = 1, LA_C2R_NATURAL = 2, LA_ADJOINT = 3 };

template <typename T>
struct LastAxisArgs {
    const cx<T> *src;  // packed (STEP, R2C_NATURAL, ADJOINT) or natural (C2R_NATURAL) input
    cx<T> *dst;        // packed (STEP, C2R_NATURAL, ADJOINT: mu) or natural (R2C_NATURAL) output
    cx<T> *dst2;       // ADJOINT: nu
    cx<T> *state;      // STEP: native state, updated in place
    int64_t nrows;
    int M;
    int W;
    int tiles_per_row;
    const cx<T> *tw;
    int lt_shift;
    ModelParams<T> mp;
    Pack pk;   // layout of the packed arrays src, dst, state (natural arrays: rows of M + 1)
    Pack pk2;  // layout of dst2 (ADJOINT's nu: plain rows of M, see x_c2r_block's EPI_ADJOINT)
};

struct SlotInfo {
    int64_t row;
    int kx;
    int partner;  // partner slot for kx == 0 pencils, -1 otherwise
    bool has_pairs;
};

// Order of the workgroups over the column tiles (3D):
//   ORD_TILE: consecutive workgroups take adjacent column tiles of one row (default);
//   ORD_ROW: consecutive workgroups take consecutive rows of one column tile (measured slightly
//            slower at 512^3);
//   ORD_XCD_ROW: workgroup b runs on XCD b mod 8 (round-robin dispatch); each XCD takes whole rows
//            (rows r with r mod 8 = its XCD, tiles in order), so that tiles whose rows are not
//            line-aligned (natural half spectrum, pitch M + 1) share their boundary lines in one
//            L2; rows past the last multiple of 8 keep the ORD_TILE order.  Used by the step's fused
//            pass too, where it measured 1.5-2 % faster than ORD_TILE (512^3 and 2048^3 FP32).
// IL: in the pair tiles, slots alternate between the two rows (slot p and its mirror p ^ 1 hold the
// same column), so that a pencil and its mirror stay in one group of adjacent slots; otherwise the
// first W/2 slots hold row k_y and the others row -k_y.
enum { ORD_TILE = 0, ORD_ROW = 1, ORD_XCD_ROW = 2 };
template <int ORD = ORD_TILE, bool IL = false>
__device__ __forceinline__ SlotInfo la_slot(int64_t nrows, int TR, int W, int p, int64_t bid)
{
    SlotInfo s;
    if (nrows == 1) {
        s.row = 0;
        s.kx = (int)bid * W + p;
        s.partner = (s.kx == 0) ? p : -1;
        s.has_pairs = (bid == 0);
        return s;
    }
    const int64_t n_normal = nrows * (TR - 1);
    if (bid < n_normal) {
        if (ORD == ORD_ROW) {
            s.row = bid % nrows;
            s.kx = (int)(1 + bid / nrows) * W + p;
        } else if (ORD == ORD_XCD_ROW && bid < (nrows - (nrows & 7)) * (TR - 1)) {
            const int64_t k = bid >> 3;
            s.row = (k / (TR - 1)) * 8 + (bid & 7);
            s.kx = (int)(1 + k % (TR - 1)) * W + p;
        } else {
            s.row = bid / (TR - 1);
            s.kx = (int)(1 + bid % (TR - 1)) * W + p;
        }
        s.partner = -1;
        s.has_pairs = false;
        return s;
    }
    // pair tiles: k in [0, nrows) takes pair i (rows i and -i; i = 0: rows 0 and nrows / 2) and half
    // h of column tile 0.  In whole groups of 16 the two halves of a pair are 8 apart (k and k + 8
    // run on one XCD under round-robin dispatch), so the lines they share meet in one L2 instead of
    // being fetched by two XCDs; a last incomplete group takes the halves in turn.
    const int64_t k = bid - n_normal, full = nrows - nrows % 16;
    const int64_t i = k < full ? ((k >> 4) << 3) + (k & 7) : (k >> 1);
    const int h = (int)(k < full ? ((k >> 3) & 1) : (k & 1)), hw = W >> 1;
    const int64_t ra = (i == 0) ? 0 : i, rb = (i == 0) ? nrows / 2 : nrows - i;
    if constexpr (IL) {
        const bool first = (p & 1) == 0;
        s.row = first ? ra : rb;
        s.kx = h * hw + (p >> 1);
        s.partner = (s.kx == 0) ? ((i == 0) ? p : (p ^ 1)) : -1;
    } else {
        const bool first = p < hw;
        s.row = first ? ra : rb;
        s.kx = h * hw + (first ? p : p - hw);
        s.partner = (s.kx == 0) ? ((i == 0) ? p : (first ? p + hw : p - hw)) : -1;
    }
    s.has_pairs = (h == 0);
    return s;
}

// G > 1 (STEP only): the pencils form G groups of WMAX / G adjacent slots that take turns in an LDS
// area of L * WMAX / G values (see fft_stages); pair tiles then interleave their two rows.
template <typename T, class PL, int WMAX, int MODE, bool PF = true, int ORD = ORD_TILE, bool NT = false, int G = 1>
__device__ __forceinline__ void last_axis_block(const LastAxisArgs<T> &a, int64_t bid, cx<T> *sh)
{
    static_assert(G == 1 || MODE == LA_STEP, "grouped LDS only in the step");
    static_assert(WMAX % G == 0 && (G == 1 || (WMAX / G) % 2 == 0), "groups must hold whole pairs");
    constexpr int L = PL::L, Tp = PL::Tp, Rmax = PL::Rmax, GW = WMAX / G;
    constexpr bool IL = G > 1;
    using PR = typename PL::Reverse;  // inverse schedule: its first radix is PL's last
    constexpr int Rl = PL::last;
    const int tid = threadIdx.x, p = tid % WMAX, t = tid / WMAX, grp = p / GW;
    const int W = a.W;
    const int64_t nrows = a.nrows, M = a.M;
    const SlotInfo si = la_slot<ORD, IL>(nrows, a.tiles_per_row, W, p < W ? p : 0, bid);
    const bool valid = p < W && si.kx < M;  // the last column tile of a row may be partial
    auto lds = [&](int e) -> cx<T> & { return sh[e * GW + p % GW]; };
    // Element e = t + k of this lane's pencil in a packed array lies at pk.at(t, row, kx) + k estride
    // (k a multiple of the layout's block size Z, which the launcher checks).  The address is split
    // into a wave-uniform part (the tile origin, the wave's first t, and k * estride: scalar
    // registers) and a per-lane 32-bit byte offset, so no per-element 64-bit vector arithmetic is
    // needed.
    const Pack &pk = a.pk;
    const int64_t estride = pk.e_stride();
    const SlotInfo s0 = la_slot<ORD, IL>(nrows, a.tiles_per_row, W, 0, bid);
    const int t0 = __builtin_amdgcn_readfirstlane(t);
    const int64_t uoff = pk.at(t0, s0.row, s0.kx);
    const uint32_t loff = (uint32_t)((pk.at(t, si.row, si.kx) - uoff) * (int64_t)sizeof(cx<T>));
    auto gp = [&](const cx<T> *base, int k) -> cx<T> * {
        return reinterpret_cast<cx<T> *>(
            reinterpret_cast<char *>(const_cast<cx<T> *>(base) + uoff + (int64_t)k * estride) + loff);
    };
    const ModelParams<T> &mp = a.mp;
    const T ky = mp.fk[1] * (T)signed_index(si.row, nrows);
    const T kx = mp.fk[2] * (T)si.kx;
    const T kxn = mp.fk[2] * (T)M;  // x Nyquist wavenumber
    cx<T> v[Rmax];

    if constexpr (MODE == LA_C2R_NATURAL) {
        // natural half spectrum in: fold kx = 0 and kx = M (projected) into one plane, inverse FFT
        constexpr int R0 = PR::first;
        const int64_t prow =
            (si.partner >= 0) ? la_slot<ORD>(nrows, a.tiles_per_row, W, si.partner, bid).row : 0;
        const int64_t pitch = M + 1;
#pragma unroll
        for (int b = 0; b < PL::nb(R0); ++b)
            if (PL::jok(t + b * Tp, R0))
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                const int e = t + b * Tp + r * (L / R0);
                cx<T> z = {T(0), T(0)};
                if (valid) {
                    const int64_t i0 = ((int64_t)e * nrows + si.row) * pitch;
                    if (si.partner < 0) {
                        z = a.src[i0 + si.kx];
                    } else {
                        const int ep = neg_mod<L>(e);
                        const int64_t i1 = ((int64_t)ep * nrows + prow) * pitch;
                        const cx<T> x0 = a.src[i0], x0p = a.src[i1], xn = a.src[i0 + M], xnp = a.src[i1 + M];
                        const T h = T(0.5);
                        const cx<T> P0 = {(x0.x + x0p.x) * h, (x0.y - x0p.y) * h};
                        const cx<T> PN = {(xn.x + xnp.x) * h, (xn.y - xnp.y) * h};
                        z = {P0.x - PN.y, P0.y + PN.x};
                    }
                }
                v[b * R0 + r] = z;
            }
        fft_stages<T, PR, +1>(v, t, lds, a.tw, a.lt_shift);
        if (valid) {
            constexpr int Rf = PR::last;
#pragma unroll
            for (int b = 0; b < PL::nb(Rf); ++b)
                if (PL::jok(t + b * Tp, Rf))
#pragma unroll
                for (int r = 0; r < Rf; ++r) st_grid<NT>(gp(a.dst, b * Tp + r * (L / Rf)), v[b * Rf + r]);
        }
        return;
    } else {
        // STEP with PF: the state values this thread updates are loaded before the forward FFT so
        // that their latency overlaps the FFT
        cx<T> spre[(MODE == LA_STEP && PF) ? Rmax : 1];
        if constexpr (MODE == LA_STEP && PF) {
#pragma unroll
            for (int b = 0; b < PL::nb(Rl); ++b)
                if (PL::jok(t + b * Tp, Rl))
#pragma unroll
                for (int r = 0; r < Rl; ++r)
                    spre[b * Rl + r] = valid ? ld_grid<NT>(gp(a.state, b * Tp + r * (L / Rl))) : cx<T>{T(0), T(0)};
        }
        // packed input, forward FFT
        constexpr int R0 = PL::first;
#pragma unroll
        for (int b = 0; b < PL::nb(R0); ++b)
            if (PL::jok(t + b * Tp, R0))
#pragma unroll
            for (int r = 0; r < R0; ++r)
                v[b * R0 + r] = valid ? ld_grid<NT>(gp(a.src, b * Tp + r * (L / R0))) : cx<T>{T(0), T(0)};
        fft_stages<T, PL, -1, TW_STAGE, G>(v, t, lds, a.tw, a.lt_shift, grp);
        // forward spectrum in natural order: v[b*Rl + r] = X(e), e = t + b*Tp + r*L/Rl
        auto partner_val = [&](int e) -> cx<T> { return sh[neg_mod<L>(e) * GW + si.partner % GW]; };
        auto spectrum_to_lds = [&]() {
#pragma unroll
            for (int b = 0; b < PL::nb(Rl); ++b)
                if (PL::jok(t + b * Tp, Rl))
#pragma unroll
                for (int r = 0; r < Rl; ++r) lds(t + b * Tp + r * (L / Rl)) = v[b * Rl + r];
        };

        if constexpr (MODE == LA_R2C_NATURAL || MODE == LA_ADJOINT) {
            if (si.has_pairs) {  // uniform per workgroup
                __syncthreads();
                spectrum_to_lds();
                __syncthreads();
            }
        }
        if constexpr (MODE == LA_R2C_NATURAL) {
            const int64_t pitch = M + 1;
            if (valid) {
#pragma unroll
                for (int b = 0; b < PL::nb(Rl); ++b)
                    if (PL::jok(t + b * Tp, Rl))
#pragma unroll
                    for (int r = 0; r < Rl; ++r) {
                        const int e = t + b * Tp + r * (L / Rl);
                        const int64_t i0 = ((int64_t)e * nrows + si.row) * pitch;
                        const cx<T> z = v[b * Rl + r];
                        if (si.partner < 0) {
                            a.dst[i0 + si.kx] = z;
                        } else {
                            const cx<T> zp = partner_val(e);
                            const T h = T(0.5);
                            a.dst[i0] = {(z.x + zp.x) * h, (z.y - zp.y) * h};
                            a.dst[i0 + M] = {(z.y + zp.y) * h, (zp.x - z.x) * h};
                        }
                    }
            }
            return;
        } else if constexpr (MODE == LA_STEP) {
            // Semi-implicit update.  Pencils off the folded column: S <- (S - dt q N) A(q).  Folded
            // column: the two planes X0 (q0) and XN (qN) are separated with the mirror element -k,
            // which another thread owns; the mirror's N comes from LDS now, its S in a second LDS
            // round, so no thread reads a state value that another thread has already updated.
            const T dt = mp.dt, nl = mp.nl, h = T(0.5);
            if (si.has_pairs) {  // uniform per workgroup
#pragma unroll
                for (int gg = 0; gg < G; ++gg) {
                    const bool mine = (G == 1) || (grp == gg);
                    __syncthreads();
                    if (mine) spectrum_to_lds();
                    __syncthreads();
                    if (mine && si.partner >= 0) {
#pragma unroll
                        for (int b = 0; b < PL::nb(Rl); ++b)
                            if (PL::jok(t + b * Tp, Rl))
#pragma unroll
                            for (int r = 0; r < Rl; ++r) {
                                const int e = t + b * Tp + r * (L / Rl);
                                const T kz = mp.fk[0] * (T)signed_index(e, L);
                                const cx<T> N = {v[b * Rl + r].x * nl, v[b * Rl + r].y * nl};
                                const cx<T> Np = {partner_val(e).x * nl, partner_val(e).y * nl};
                                const cx<T> N0 = {(N.x + Np.x) * h, (N.y - Np.y) * h};
                                const cx<T> NN = {(N.y + Np.y) * h, (Np.x - N.x) * h};
                                const T q0 = kz * kz + ky * ky, qn = q0 + kxn * kxn;
                                const T g0 = dt * q0 * amult(mp, q0), gn = dt * qn * amult(mp, qn);
                                // G = -(g0 N0 + i gn NN): the cubic term's share of the new value
                                v[b * Rl + r] = {-g0 * N0.x + gn * NN.y, -g0 * N0.y - gn * NN.x};
                            }
                    }
                }
            }
            if (si.partner < 0) {
#pragma unroll
                for (int b = 0; b < PL::nb(Rl); ++b)
                    if (PL::jok(t + b * Tp, Rl))
#pragma unroll
                    for (int r = 0; r < Rl; ++r) {
                        const int e = t + b * Tp + r * (L / Rl);
                        const T kz = mp.fk[0] * (T)signed_index(e, L);
                        const cx<T> N = {v[b * Rl + r].x * nl, v[b * Rl + r].y * nl};
                        cx<T> *gi = gp(a.state, b * Tp + r * (L / Rl));
                        cx<T> S;
                        if constexpr (PF)
                            S = spre[b * Rl + r];
                        else
                            S = valid ? ld_grid<NT>(gi) : cx<T>{T(0), T(0)};
                        const T q = kz * kz + ky * ky + kx * kx;
                        const T A = amult(mp, q), dq = dt * q;
                        const cx<T> Snew = {(S.x - dq * N.x) * A, (S.y - dq * N.y) * A};
                        if (valid) st_grid<NT>(gi, Snew);
                        v[b * Rl + r] = Snew;
                    }
            }
            if (si.has_pairs) {  // uniform per workgroup
#pragma unroll
                for (int gg = 0; gg < G; ++gg) {
                    const bool mine = (G == 1) || (grp == gg);
                    __syncthreads();  // every mirror N has been read
                    if (mine && si.partner >= 0 && valid) {
#pragma unroll
                        for (int b = 0; b < PL::nb(Rl); ++b)
                            if (PL::jok(t + b * Tp, Rl))
#pragma unroll
                            for (int r = 0; r < Rl; ++r) {
                                const int e = t + b * Tp + r * (L / Rl);
                                if constexpr (PF)
                                    lds(e) = spre[b * Rl + r];
                                else
                                    lds(e) = ld_grid<NT>(gp(a.state, b * Tp + r * (L / Rl)));
                            }
                    }
                    __syncthreads();
                    if (mine && si.partner >= 0) {
#pragma unroll
                        for (int b = 0; b < PL::nb(Rl); ++b)
                            if (PL::jok(t + b * Tp, Rl))
#pragma unroll
                            for (int r = 0; r < Rl; ++r) {
                                const int e = t + b * Tp + r * (L / Rl);
                                const T kz = mp.fk[0] * (T)signed_index(e, L);
                                cx<T> *gi = gp(a.state, b * Tp + r * (L / Rl));
                                cx<T> S;
                                if constexpr (PF)
                                    S = spre[b * Rl + r];
                                else
                                    S = valid ? ld_grid<NT>(gi) : cx<T>{T(0), T(0)};
                                const cx<T> Sp = partner_val(e);
                                const cx<T> S0 = {(S.x + Sp.x) * h, (S.y - Sp.y) * h};
                                const cx<T> SN = {(S.y + Sp.y) * h, (Sp.x - S.x) * h};
                                const T q0 = kz * kz + ky * ky, qn = q0 + kxn * kxn;
                                const T A0 = amult(mp, q0), AN = amult(mp, qn);
                                const cx<T> Gt = v[b * Rl + r];
                                // A0 S0 + i AN SN + G
                                const cx<T> Snew = {A0 * S0.x - AN * SN.y + Gt.x, A0 * S0.y + AN * SN.x + Gt.y};
                                if (valid) st_grid<NT>(gi, Snew);
                                v[b * Rl + r] = Snew;
                            }
                    }
                }
            }
            fft_stages<T, PR, +1, TW_STAGE, G>(v, t, lds, a.tw, a.lt_shift, grp);
            if (valid) {
                constexpr int Rf = PR::last;
#pragma unroll
                for (int b = 0; b < PL::nb(Rf); ++b)
                    if (PL::jok(t + b * Tp, Rf))
#pragma unroll
                    for (int r = 0; r < Rf; ++r) st_grid<NT>(gp(a.dst, b * Tp + r * (L / Rf)), v[b * Rf + r]);
            }
        } else if constexpr (MODE == LA_ADJOINT) {
            cx<T> w[Rmax];
#pragma unroll
            for (int b = 0; b < PL::nb(Rl); ++b)
                if (PL::jok(t + b * Tp, Rl))
#pragma unroll
                for (int r = 0; r < Rl; ++r) {
                    const int e = t + b * Tp + r * (L / Rl);
                    const T kz = mp.fk[0] * (T)signed_index(e, L);
                    const cx<T> z = v[b * Rl + r];
                    cx<T> mu, nu;
                    if (si.partner < 0) {
                        const T q = kz * kz + ky * ky + kx * kx;
                        const T A = amult(mp, q);
                        mu = {z.x * A, z.y * A};
                        nu = {mu.x * q, mu.y * q};
                    } else {
                        const cx<T> zp = partner_val(e);
                        const T h = T(0.5);
                        const cx<T> U = {(z.x + zp.x) * h, (z.y - zp.y) * h};
                        const cx<T> V = {(z.y + zp.y) * h, (zp.x - z.x) * h};
                        const T q0 = kz * kz + ky * ky, qn = q0 + kxn * kxn;
                        const T A0 = amult(mp, q0), AN = amult(mp, qn);
                        const cx<T> mU = {U.x * A0, U.y * A0}, mV = {V.x * AN, V.y * AN};
                        mu = {mU.x - mV.y, mU.y + mV.x};
                        nu = {mU.x * q0 - mV.y * qn, mU.y * q0 + mV.x * qn};
                    }
                    v[b * Rl + r] = mu;
                    w[b * Rl + r] = nu;
                }
            constexpr int Rf = PR::last;
            const int64_t uoff2 = a.pk2.at(t0, s0.row, s0.kx), estride2 = a.pk2.e_stride();
            const uint32_t loff2 = (uint32_t)((a.pk2.at(t, si.row, si.kx) - uoff2) * (int64_t)sizeof(cx<T>));
            auto gp2 = [&](cx<T> *base, int k) -> cx<T> * {
                return reinterpret_cast<cx<T> *>(reinterpret_cast<char *>(base + uoff2 + (int64_t)k * estride2) + loff2);
            };
            fft_stages<T, PR, +1>(v, t, lds, a.tw, a.lt_shift);
            if (valid) {
#pragma unroll
                for (int b = 0; b < PL::nb(Rf); ++b)
                    if (PL::jok(t + b * Tp, Rf))
#pragma unroll
                    for (int r = 0; r < Rf; ++r) *gp(a.dst, b * Tp + r * (L / Rf)) = v[b * Rf + r];
            }
            fft_stages<T, PR, +1>(w, t, lds, a.tw, a.lt_shift);
            if (valid) {
#pragma unroll
                for (int b = 0; b < PL::nb(Rf); ++b)
                    if (PL::jok(t + b * Tp, Rf))
#pragma unroll
                    for (int r = 0; r < Rf; ++r) *gp2(a.dst2, b * Tp + r * (L / Rf)) = w[b * Rf + r];
            }
        }
    }
}

template <typename T, class PL, int WMAX, int MODE, int OCC = 1, bool PF = true, int ORD = ORD_TILE, bool NT = false,
          int G = 1>
__global__ __launch_bounds__(WMAX *PL::Tp, OCC) void last_axis_kernel(LastAxisArgs<T> a)
{
    __shared__ cx<T> sh[PL::L * WMAX / G];
    last_axis_block<T, PL, WMAX, MODE, PF, ORD, NT, G>(a, blockIdx.x, sh);
}

// ------------------------------------------------------------------------------------------------
// Hydrodynamic PFC: pointwise operations on packed spectra (layout: element (e, row, kx) at
// (e nrows + row) M + kx; column kx = 0 holds the planes kx = 0 and kx = M as X0 + i XN).

__device__ __forceinline__ double hy_corr(const HydroArgs &h, double q)
{
    const double a = (1.0 - q) * (1.0 - q);
    if (h.model == 0) return a;
    const double b = h.q1sq - q;
    return a * (b * b + h.R1);
}

enum { HY_PSI = 0, HY_MU = 1, HY_VEL = 2 };

// The update of one mode for its q, with real coefficients (so it maps Hermitian planes to
// Hermitian planes):
//   HY_PSI: S <- (S - dt q nl N - dt B) / (1 + dt q (r + L(q)))    (out = S, x0 = N, x1 = B)
//   HY_MU:  A <- nl A + (r + L(q)) S                                 (out = A, x0 = S)
//   HY_VEL: V <- (V - c G(q) B) / (1 + c Gamma q), G = exp(-a0^2 q/2) (out = V, x0 = B)
template <int OP>
__device__ __forceinline__ void hy_mode(const HydroArgs &h, double q, double o[2], const double a[2], const double b[2])
{
    if constexpr (OP == HY_PSI) {
        const double den = 1.0 + h.dt * q * (h.r + hy_corr(h, q)), f = -h.dt * q * h.nl;
        for (int c = 0; c < 2; ++c) o[c] = (o[c] + f * a[c] - h.dt * b[c]) / den;
    } else if constexpr (OP == HY_MU) {
        const double m = h.r + hy_corr(h, q);
        for (int c = 0; c < 2; ++c) o[c] = h.nl * o[c] + m * a[c];
    } else {
        const double g = h.c * exp(-0.5 * h.a0 * h.a0 * q), den = 1.0 + h.c * h.gamma * q;
        for (int c = 0; c < 2; ++c) o[c] = (o[c] - g * a[c]) / den;
    }
}

// Applies hy_mode to every mode of a packed spectrum, in place on `out`.  On the folded column a
// thread takes the pair (k, -k): it separates X0 and XN of every operand with the mirror element,
// updates each plane with its own q (q0 or q0 + kx_Nyquist^2) and writes both elements.
template <typename T, int OP>
__global__ __launch_bounds__(256) void spec_update_kernel(cx<T> *out, const cx<T> *__restrict__ x0,
                                                          const cx<T> *__restrict__ x1, int64_t L, int64_t nrows,
                                                          int64_t M, HydroArgs h, Pack pk)
{
    const int64_t n = L * nrows * M;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t kx = i % M, rest = i / M, row = rest % nrows, e = rest / nrows;
        const int64_t j = pk.at(e, row, kx);  // i: logical index, j: its place in memory
        const double kz = h.fk[0] * signed_index(e, L), ky = h.fk[1] * signed_index(row, nrows);
        const cx<T> zx1 = x1 ? x1[j] : cx<T>{T(0), T(0)};
        if (kx != 0) {
            const double kk = h.fk[2] * (double)kx, q = kz * kz + ky * ky + kk * kk;
            double o[2] = {(double)out[j].x, (double)out[j].y}, a[2] = {(double)x0[j].x, (double)x0[j].y},
                   b[2] = {(double)zx1.x, (double)zx1.y};
            hy_mode<OP>(h, q, o, a, b);
            out[j] = {(T)o[0], (T)o[1]};
            continue;
        }
        const int64_t em = (L - e) % L, rm = (nrows - row) % nrows;
        const int64_t im = (em * nrows + rm) * M;
        if (im < i) continue;  // the pair is updated by the thread of its lower (logical) index
        const int64_t jm = pk.at(em, rm, 0);
        const cx<T> mx1 = x1 ? x1[jm] : cx<T>{T(0), T(0)};
        const cx<T> Z[3] = {out[j], x0[j], zx1}, Zm[3] = {out[jm], x0[jm], mx1};
        double p0[3][2], pn[3][2];  // X0 and XN of each operand at k
        for (int j = 0; j < 3; ++j) {
            p0[j][0] = 0.5 * ((double)Z[j].x + (double)Zm[j].x);
            p0[j][1] = 0.5 * ((double)Z[j].y - (double)Zm[j].y);
            pn[j][0] = 0.5 * ((double)Z[j].y + (double)Zm[j].y);
            pn[j][1] = 0.5 * ((double)Zm[j].x - (double)Z[j].x);
        }
        const double kn = h.fk[2] * (double)M, q0 = kz * kz + ky * ky, qn = q0 + kn * kn;
        hy_mode<OP>(h, q0, p0[0], p0[1], p0[2]);
        hy_mode<OP>(h, qn, pn[0], pn[1], pn[2]);
        // Y = Y0 + i YN at k; at -k the planes are conjugated: conj Y0 + i conj YN
        out[j] = {(T)(p0[0][0] - pn[0][1]), (T)(p0[0][1] + pn[0][0])};
        if (im != i) out[jm] = {(T)(p0[0][0] + pn[0][1]), (T)(pn[0][0] - p0[0][1])};
    }
}

// ------------------------------------------------------------------------------------------------
// Last axis of the 3D r2c into the natural half spectrum (rows of M + 1 values), by line-aligned
// chunks.  The output plane (nrows rows of M + 1) is cut into chunks of C = 128 / sizeof(cx)
// consecutive values; workgroup c owns output positions f = cC .. cC + C - 1 of every plane, i.e.
// one whole 128-byte line per plane (requires nrows (M + 1) % C == 0 and M >= C), so no line is
// written by two workgroups.  Slot p computes the pencil of position f: row f / (M + 1), column
// kx = f % (M + 1).  For 1 <= kx < M that is packed column kx; kx = 0 and kx = M are the two planes
// folded into packed column 0, separated with the mirror pencil (row -k_y, element -k_z), which a
// second round transforms: X0 = (Z(k) + conj Z(-k)) / 2, XM = -i (Z(k) - conj Z(-k)) / 2.  A chunk
// holds at most two such slots; the second round runs only in chunks that have one.  The reads of
// packed columns are not line-aligned; chunks that share input lines run on one XCD.
template <typename T, class PL, int C, int G, bool NT = false>
__global__ __launch_bounds__(C *PL::Tp) void r2c_natural_chunk_kernel(const cx<T> *__restrict__ src,
                                                                      cx<T> *__restrict__ dst, int64_t nrows, int M,
                                                                      const cx<T> *__restrict__ tw, int lt_shift,
                                                                      Pack pk)
{
    constexpr int L = PL::L, Tp = PL::Tp, Rmax = PL::Rmax, R0 = PL::first, Rl = PL::last, GW = C / G;
    __shared__ cx<T> sh[L * GW];
    const int tid = threadIdx.x, p = tid % C, t = tid / C, grp = p / GW;
    auto lds = [&](int e) -> cx<T> & { return sh[e * GW + p % GW]; };
    const int64_t pitch = (int64_t)M + 1, plane = nrows * pitch, nchunks = plane / C;
    const int64_t chunk = xcd_tile_order(blockIdx.x, nchunks, 16);
    const int64_t f = chunk * C + p;
    const int64_t row = f / pitch;
    const int kx = (int)(f - row * pitch);
    const bool fold = (kx == 0 || kx == M);
    const int64_t estride = pk.e_stride();  // element steps k below are multiples of the layout's block
    cx<T> v[Rmax];
    // first sweep: own pencil (folded slots: packed column 0 of this row)
    {
        const cx<T> *col = src + pk.at(t, row, fold ? 0 : kx);
#pragma unroll
        for (int b = 0; b < PL::nb(R0); ++b)
            if (PL::jok(t + b * Tp, R0))
#pragma unroll
            for (int r = 0; r < R0; ++r) v[b * R0 + r] = col[(int64_t)(b * Tp + r * (L / R0)) * estride];
    }
    fft_stages<T, PL, -1, TW_STAGE, G>(v, t, lds, tw, lt_shift, grp);
    if (!fold) {
#pragma unroll
        for (int b = 0; b < PL::nb(Rl); ++b)
            if (PL::jok(t + b * Tp, Rl))
#pragma unroll
            for (int r = 0; r < Rl; ++r) st_grid<NT>(&dst[(int64_t)(t + b * Tp + r * (L / Rl)) * plane + f], v[b * Rl + r]);
    }
    if (!__syncthreads_or(fold)) return;  // uniform: the chunk has no folded slot
    // second sweep: mirror pencils of the folded slots
    cx<T> z[Rmax];
#pragma unroll
    for (int i = 0; i < Rmax; ++i) z[i] = v[i];
    {
        const int64_t mrow = (nrows - row) % nrows;
        const cx<T> *col = src + pk.at(t, mrow, 0);
#pragma unroll
        for (int b = 0; b < PL::nb(R0); ++b)
            if (PL::jok(t + b * Tp, R0))
#pragma unroll
            for (int r = 0; r < R0; ++r)
                v[b * R0 + r] = fold ? col[(int64_t)(b * Tp + r * (L / R0)) * estride] : cx<T>{T(0), T(0)};
    }
    fft_stages<T, PL, -1, TW_STAGE, G>(v, t, lds, tw, lt_shift, grp);
    const T h = T(0.5);
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
        const bool mine = (G == 1) || (grp == gg);
        __syncthreads();
        if (mine) {
#pragma unroll
            for (int b = 0; b < PL::nb(Rl); ++b)
                if (PL::jok(t + b * Tp, Rl))
#pragma unroll
                for (int r = 0; r < Rl; ++r) lds(t + b * Tp + r * (L / Rl)) = v[b * Rl + r];
        }
        __syncthreads();
        if (mine && fold) {
#pragma unroll
            for (int b = 0; b < PL::nb(Rl); ++b)
                if (PL::jok(t + b * Tp, Rl))
#pragma unroll
                for (int r = 0; r < Rl; ++r) {
                    const int e = t + b * Tp + r * (L / Rl);
                    const cx<T> a = z[b * Rl + r], m = lds(neg_mod<L>(e));
                    const cx<T> out = (kx == 0) ? cx<T>{(a.x + m.x) * h, (a.y - m.y) * h}
                                                : cx<T>{(a.y + m.y) * h, (m.x - a.x) * h};
                    st_grid<NT>(&dst[(int64_t)e * plane + f], out);
                }
        }
    }
}

// ------------------------------------------------------------------------------------------------
// Reductions (FP64 accumulation, fixed grid and order: deterministic).

// partial[block] = sum of x over a grid-stride range.
template <typename T>
__global__ __launch_bounds__(256) void sum_kernel(const T *__restrict__ x, int64_t n, double *partial)
{
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc += (double)x[i];
    __shared__ double red[4];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// state[0].x = (T) sum(partial[0..np)) -- the mass mode from an FP64 sum of the field.
template <typename T>
__global__ void set_mass_kernel(const double *partial, int np, cx<T> *state)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < np; ++i) s += partial[i];
        state[0].x = (T)s;
    }
}

// *acc += coef * sum(partial[0..np))
__global__ void accumulate_kernel(const double *partial, int np, double coef, double *acc);

// Spectral quadratic part of the energy: sum over the full spectrum of (r + L(q)) |psi_hat|^2,
// from the native state (FP64 throughout).  Geometry as in the last-axis pass.
template <typename T>
__global__ __launch_bounds__(256) void energy_spec_kernel(const cx<T> *__restrict__ state, int64_t L, int64_t nrows,
                                                          int64_t M, double fk0, double fk1, double fk2, double r,
                                                          double q1sq, double R1, int model, double *partial, Pack pk)
{
    const int64_t n = L * nrows * M;
    auto corr = [&](double q) {
        double a = (1.0 - q) * (1.0 - q);
        if (model == 0) return a;
        double b = q1sq - q;
        return a * (b * b + R1);
    };
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t kx = i % M, rest = i / M, row = rest % nrows, e = rest / nrows;
        const double kz = fk0 * signed_index(e, L), ky = fk1 * signed_index(row, nrows);
        const cx<T> s = state[pk.at(e, row, kx)];
        if (kx != 0) {
            const double k = fk2 * (double)kx, q = kz * kz + ky * ky + k * k;
            acc += 2.0 * (r + corr(q)) * ((double)s.x * s.x + (double)s.y * s.y);
        } else {
            const int64_t ep = (L - e) % L, rp = (nrows - row) % nrows;
            const cx<T> sp = state[pk.at(ep, rp, 0)];
            const double ax = 0.5 * ((double)s.x + sp.x), ay = 0.5 * ((double)s.y - sp.y);
            const double bx = 0.5 * ((double)s.y + sp.y), by = 0.5 * ((double)sp.x - s.x);
            const double q0 = kz * kz + ky * ky, kn = fk2 * (double)M, qn = q0 + kn * kn;
            acc += (r + corr(q0)) * (ax * ax + ay * ay) + (r + corr(qn)) * (bx * bx + by * by);
        }
    }
    __shared__ double red[4];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <typename T>
__global__ __launch_bounds__(256) void quartic_kernel(const T *__restrict__ psi, int64_t n, double *partial)
{
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = (double)psi[i] * (double)psi[i];
        acc += 0.25 * v * v;
    }
    __shared__ double red[4];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// out[0] = dV (sum(ps)/(2N) + sum(pq)), out[1] = state[0].x / N.
template <typename T>
__global__ void energy_final_kernel(const double *ps, const double *pq, int np, double dV, double ntot,
                                    const cx<T> *state, double *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int i = 0; i < np; ++i) a += ps[i];
        for (int i = 0; i < np; ++i) b += pq[i];
        out[0] = dV * (a / (2.0 * ntot) + b);
        out[1] = (double)state[0].x / ntot;
    }
}

// Native state -> natural half spectrum [L][nrows][M+1].
template <typename T>
__global__ __launch_bounds__(256) void export_kernel(const cx<T> *__restrict__ state, cx<T> *__restrict__ out,
                                                     int64_t L, int64_t nrows, int64_t M, Pack pk)
{
    const int64_t n = L * nrows * (M + 1);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t kx = i % (M + 1), rest = i / (M + 1), row = rest % nrows, e = rest / nrows;
        if (kx > 0 && kx < M) {
            out[i] = state[pk.at(e, row, kx)];
        } else {
            const int64_t ep = (L - e) % L, rp = (nrows - row) % nrows;
            const cx<T> s = state[pk.at(e, row, 0)], sp = state[pk.at(ep, rp, 0)];
            const T h = T(0.5);
            out[i] = (kx == 0) ? cx<T>{(s.x + sp.x) * h, (s.y - sp.y) * h} : cx<T>{(s.y + sp.y) * h, (sp.x - s.x) * h};
        }
    }
}

}  // namespace pfc
