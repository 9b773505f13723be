// apfc.hpp -- kernels of the complex-amplitude form of the PFC model (the amplitude extension
// named at the end of the paper's multiphysics section).  The density is expanded as
// psi = sum_j eta_j e^{i k_j.r} + c.c. over N principal reciprocal-lattice vectors k_j; each
// complex amplitude follows
//     d_t eta_j = -|k_j|^2 [ (dB + Bx (1 - |k_j|^2 + G_j)^2) eta_j + N_j ],   G_j = lap + 2 i k_j.grad,
// N_j the resonant part of -t psi^2 + v psi^3 at k_j, stepped like Listing 1's update; in Fourier
// space 1 - |k_j|^2 + G_j = 1 - |q + k_j|^2:
//     eta_hat_j <- (eta_hat_j - dt |k_j|^2 FFT(N_j)) / (1 + dt |k_j|^2 (dB + Bx (1 - |q + k_j|^2)^2)).
// Fields are N complex grids back to back, C order (axis 0 slowest, x contiguous); spectra in
// natural FFT order.  Kernels here: the pointwise nonlinearity, complex FFTs of contiguous rows
// (x pass), and the fused last-axis pass (forward FFT, update of every amplitude, inverse FFT).
#pragma once

#include "apfc_launch.hpp"
#include "kernels.hpp"

namespace pfc {

template <typename T>
__device__ __forceinline__ T apfc_coef(const ApfcTerm &m)
{
    if constexpr (sizeof(T) == 4)
        return m.coef32;
    else
        return m.coef;
}

// Amplitude s of this thread's point from its LDS slots (field f at slot f * stride).
template <typename T>
__device__ __forceinline__ cx<T> apfc_pick(const cx<T> *mine, int s, int stride)
{
    const int f = (s > 0 ? s : -s) - 1;
    const cx<T> z = mine[f * stride];
    return s > 0 ? z : cx<T>{z.x, -z.y};
}

// out_j = N_j at every point, for all fields.  One point per thread: the thread's N amplitudes sit
// in LDS (a runtime-indexed register array would live in scratch memory).  The ordered triples that
// are a permutation of (j, i, -i) are resonant on every lattice (6 orders for i != j, 3 for i = j);
// their sum is c3 (A^2 - |eta_j|^2) eta_j with A^2 = 2 sum_i |eta_i|^2 and c3 = 3v.  The remaining
// products terms[off[j] .. off[j+1]) are summed one by one.
constexpr int kApfcThreads = 128;
// PPT points per thread (PPT consecutive groups of kApfcThreads points per workgroup): each term of
// the table is then read once for PPT points.  Dynamic LDS: nf * PPT * kApfcThreads * sizeof(cx<T>).
template <typename T, int PPT>
__global__ __launch_bounds__(kApfcThreads) void apfc_nonlin_kernel(const cx<T> *__restrict__ eta,
                                                                   cx<T> *__restrict__ out, int64_t P, int nf,
                                                                   const ApfcTerm *__restrict__ terms,
                                                                   const int *__restrict__ off, T c3)
{
    constexpr int S = PPT * kApfcThreads;  // LDS stride between fields
    extern __shared__ __align__(16) unsigned char apfc_lds[];
    cx<T> *mine[PPT];
    int64_t idx[PPT];
    bool valid[PPT];
    T A2[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        mine[q] = reinterpret_cast<cx<T> *>(apfc_lds) + q * kApfcThreads + threadIdx.x;
        idx[q] = (int64_t)blockIdx.x * S + q * kApfcThreads + threadIdx.x;
        valid[q] = idx[q] < P;
        A2[q] = T(0);
    }
    // loads in groups of 8 fields, all in flight before the first one is used
    for (int f0 = 0; f0 < nf; f0 += 8) {
        cx<T> z[PPT][8];
#pragma unroll
        for (int q = 0; q < PPT; ++q)
#pragma unroll
            for (int u = 0; u < 8; ++u)
                z[q][u] = (valid[q] && f0 + u < nf) ? eta[(int64_t)(f0 + u) * P + idx[q]] : cx<T>{T(0), T(0)};
#pragma unroll
        for (int q = 0; q < PPT; ++q)
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (f0 + u < nf) {
                    mine[q][(f0 + u) * S] = z[q][u];
                    A2[q] += z[q][u].x * z[q][u].x + z[q][u].y * z[q][u].y;
                }
    }
    // each thread reads back only its own slots: no barrier needed
    for (int j = 0; j < nf; ++j) {
        // the triples eta_j eta_i conj(eta_i), resonant on every lattice, summed in closed form
        cx<T> acc[PPT];
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const cx<T> zj = mine[q][j * S];
            const T g = c3 * (T(2) * A2[q] - (zj.x * zj.x + zj.y * zj.y));
            acc[q] = {g * zj.x, g * zj.y};
        }
        const int m1 = off[j + 1];
        for (int m = off[j]; m < m1; ++m) {
            const ApfcTerm tm = terms[m];
            const T c = apfc_coef<T>(tm);
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                cx<T> p = cmul(apfc_pick(mine[q], tm.a, S), apfc_pick(mine[q], tm.b, S));
                if (tm.c != 0) p = cmul(p, apfc_pick(mine[q], tm.c, S));
                acc[q] = {acc[q].x + c * p.x, acc[q].y + c * p.y};
            }
        }
#pragma unroll
        for (int q = 0; q < PPT; ++q)
            if (valid[q]) out[(int64_t)j * P + idx[q]] = acc[q];
    }
}

// Complex FFT of contiguous rows of length L (the x pass), in place or out of place, times
// `scale` on the way out.  ROWS rows per workgroup, Tp threads per row; coalesced loads and
// stores (neighbouring threads take neighbouring elements).
template <typename T, class PL, int ROWS, int DIR, bool NT = false>
__global__ __launch_bounds__(ROWS *PL::Tp) void apfc_row_kernel(const cx<T> *in, cx<T> *out, int64_t nrows,
                                                               const cx<T> *__restrict__ tw, int lt_shift, T scale)
{
    constexpr int L = PL::L, Tp = PL::Tp, R0 = PL::first, Rl = PL::last, Rmax = PL::Rmax;
    __shared__ cx<T> sh[ROWS * L];
    const int tid = threadIdx.x, p = tid / Tp, t = tid - p * Tp;
    const int64_t row = (int64_t)blockIdx.x * ROWS + p;
    const bool valid = row < nrows;
    const cx<T> *src = in + (valid ? row : 0) * L;
    cx<T> v[Rmax];
#pragma unroll
    for (int b = 0; b < PL::nb(R0); ++b)
        if (PL::jok(t + b * Tp, R0))
#pragma unroll
        for (int r = 0; r < R0; ++r)
            v[b * R0 + r] = valid ? ld_grid<NT>(&src[t + b * Tp + r * (L / R0)]) : cx<T>{T(0), T(0)};
    auto lds = [&](int e) -> cx<T> & { return sh[p * L + e]; };
    fft_stages<T, PL, DIR>(v, t, lds, tw, lt_shift);
    if (valid) {
        cx<T> *dst = out + row * L;
#pragma unroll
        for (int b = 0; b < PL::nb(Rl); ++b)
            if (PL::jok(t + b * Tp, Rl))
#pragma unroll
            for (int r = 0; r < Rl; ++r) {
                const cx<T> z = v[b * Rl + r];
                st_grid<NT>(&dst[t + b * Tp + r * (L / Rl)], cx<T>{z.x * scale, z.y * scale});
            }
    }
}

// signed index of Fourier mode i on an axis of length n in numpy's fftfreq order (Nyquist negative)
__device__ __forceinline__ int fft_freq(int64_t i, int64_t n) { return (int)(2 * i < n ? i : i - n); }

// Fused last-axis pass of the amplitude step (arguments in apfc_launch.hpp): completes the forward
// FFT of FFT(N_f) along this axis, updates the state in place and writes the inverse FFT along this
// axis of the new state to dst.
template <typename T, class PL, int WMAX, bool PF, int G>
__global__ __launch_bounds__(WMAX *PL::Tp) void apfc_last_step_kernel(ApfcStepArgs<T> a)
{
    static_assert(WMAX % G == 0, "groups of whole pencils");
    constexpr int L = PL::L, Tp = PL::Tp, Rmax = PL::Rmax, R0 = PL::first, Rl = PL::last, GW = WMAX / G;
    using PR = typename PL::Reverse;
    __shared__ cx<T> sh[L * WMAX / G];
    const int tid = threadIdx.x, p = tid % WMAX, t = tid / WMAX, grp = p / GW;
    const int64_t bid = blockIdx.x;
    const int f = (int)(bid / a.tiles);
    const int64_t col = (bid - (int64_t)f * a.tiles) * a.W + p;
    const bool valid = p < a.W && col < a.ncols;
    const int64_t base = (int64_t)f * a.fstride + (valid ? col : 0);
    auto at = [&](cx<T> *g, int e) -> cx<T> * { return g + base + (int64_t)e * a.ncols; };
    auto lds = [&](int e) -> cx<T> & { return sh[e * GW + p % GW]; };

    cx<T> spre[PF ? Rmax : 1];
    if constexpr (PF) {
#pragma unroll
        for (int b = 0; b < PL::nb(Rl); ++b)
            if (PL::jok(t + b * Tp, Rl))
#pragma unroll
            for (int r = 0; r < Rl; ++r)
                spre[b * Rl + r] = valid ? *at(a.state, t + b * Tp + r * (L / Rl)) : cx<T>{T(0), T(0)};
    }
    cx<T> v[Rmax];
#pragma unroll
    for (int b = 0; b < PL::nb(R0); ++b)
        if (PL::jok(t + b * Tp, R0))
#pragma unroll
        for (int r = 0; r < R0; ++r)
            v[b * R0 + r] = valid ? *at(const_cast<cx<T> *>(a.src), t + b * Tp + r * (L / R0)) : cx<T>{T(0), T(0)};
    fft_stages<T, PL, -1, TW_STAGE, G>(v, t, lds, a.tw, a.lt_shift, grp);

    // per-pencil part of the operator: the two other axes
    const int64_t k1i = valid ? col / a.nx : 0, kxi = valid ? col - k1i * a.nx : 0;
    const T q1 = a.fk[1] * (T)fft_freq(k1i, a.n1), qx = a.fk[2] * (T)fft_freq(kxi, a.nx);
    const T k0 = a.kv[f][0], kq12 = a.kv[f][1] * q1 + a.kv[f][2] * qx, q12 = q1 * q1 + qx * qx;
    const T dq = a.dt * a.kk[f], c1 = T(1) - a.kk[f];
#pragma unroll
    for (int b = 0; b < PL::nb(Rl); ++b)
        if (PL::jok(t + b * Tp, Rl))
#pragma unroll
        for (int r = 0; r < Rl; ++r) {
            const int e = t + b * Tp + r * (L / Rl);
            const T q0 = a.fk[0] * (T)fft_freq(e, L);
            const T Gj = c1 - (q0 * q0 + q12 + T(2) * (k0 * q0 + kq12));  // 1 - |q + k_f|^2
            const T inv = T(1) / (T(1) + dq * (a.dB + a.Bx * Gj * Gj));
            cx<T> S;
            if constexpr (PF)
                S = spre[b * Rl + r];
            else
                S = valid ? *at(a.state, e) : cx<T>{T(0), T(0)};
            const cx<T> N = v[b * Rl + r];
            const cx<T> Snew = {(S.x - dq * N.x) * inv, (S.y - dq * N.y) * inv};
            if (valid) *at(a.state, e) = Snew;
            v[b * Rl + r] = Snew;
        }
    fft_stages<T, PR, +1, TW_STAGE, G>(v, t, lds, a.tw, a.lt_shift, grp);
    if (valid) {
        constexpr int Rf = PR::last;
#pragma unroll
        for (int b = 0; b < PL::nb(Rf); ++b)
            if (PL::jok(t + b * Tp, Rf))
#pragma unroll
            for (int r = 0; r < Rf; ++r) *at(a.dst, t + b * Tp + r * (L / Rf)) = v[b * Rf + r];
    }
}

}  // namespace pfc
