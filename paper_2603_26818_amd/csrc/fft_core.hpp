// fft_core.hpp -- device building blocks of the pencil FFTs (gfx950, wave64).
//
// A length-L complex FFT of one "pencil" is done by Tp = L / Rmax threads with a Stockham
// autosort schedule: stage s has radix R_s; each thread runs Rmax / R_s radix-R_s butterflies from
// registers, and the stages exchange data through LDS.  The first stage reads its inputs straight
// from the caller (global memory, coalesced) and the last stage leaves its outputs in registers in
// natural order, so an FFT costs (stages - 1) LDS round trips and no extra HBM traffic.
//
// Stage s with radix R after the radices before it multiply to Ns (Ns = 1 for the first stage):
//   thread butterfly j in [0, L/R):  a_r = x[j + r L/R] * W_{Ns R}^{(j mod Ns) r},  r < R
//                                    y   = DFT_R(a)
//                                    out[(j / Ns) Ns R + (j mod Ns) + r Ns] = y_r
// which after the last stage (Ns R = L) writes element j + r L/R.  Twiddles come from the buffer
// described in types.hpp (computed on the host): either the table W_Lt^e = exp(-2 pi i e / Lt),
// e < Lt, for a power of two Lt >= L (TW_LT), or the per-stage tables stored after it, where the
// R - 1 twiddles of a butterfly are adjacent and need no index arithmetic (TW_STAGE).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "types.hpp"

namespace pfc {

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.x, -a.y}; }
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
// i * a
template <typename T>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) { return {-a.y, a.x}; }
// -i * a
template <typename T>
__device__ __forceinline__ cx<T> mul_mi(cx<T> a) { return {a.y, -a.x}; }

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// cos and sin of 2 pi k / 16 (k = 0..4), to more digits than double holds.
__host__ __device__ constexpr double c16(int k)
{
    return k == 0 ? 1.0
         : k == 1 ? 0.92387953251128675612818318939678828682
         : k == 2 ? 0.70710678118654752440084436210484903928
         : k == 3 ? 0.38268343236508977172845998403039886676
                  : 0.0;
}
// cos(2 pi k / 16) for any k, by symmetry of the table above.
__host__ __device__ constexpr double cos16(int k)
{
    k &= 15;
    return k <= 4 ? c16(k) : k <= 8 ? -c16(8 - k) : k <= 12 ? -c16(k - 8) : c16(16 - k);
}
__host__ __device__ constexpr double sin16(int k) { return cos16(k - 4); }

// a * exp(DIR * 2 pi i K / R), DIR = -1 (forward) or +1 (inverse), R <= 16.
template <typename T, int R, int K, int DIR>
__device__ __forceinline__ cx<T> rot(cx<T> a)
{
    constexpr int k16 = ((K * 16) / R) & 15;
    if constexpr (k16 == 0) {
        return a;
    } else if constexpr (k16 == 8) {
        return {-a.x, -a.y};
    } else if constexpr (k16 == 4) {
        return DIR > 0 ? mul_i(a) : mul_mi(a);
    } else if constexpr (k16 == 12) {
        return DIR > 0 ? mul_mi(a) : mul_i(a);
    } else {
        constexpr T c = (T)cos16(k16);
        constexpr T s = (T)(DIR * sin16(k16));
        return {a.x * c - a.y * s, a.x * s + a.y * c};
    }
}

// In-register DFT of size R (power of two <= 16), natural order in and out.  Radix-2 decimation
// in time, fully unrolled.
template <typename T, int R, int DIR>
__device__ __forceinline__ void dft(cx<T> *v)
{
    if constexpr (R == 2) {
        cx<T> a = v[0], b = v[1];
        v[0] = a + b;
        v[1] = a - b;
    } else if constexpr (R > 2) {
        cx<T> e[R / 2], o[R / 2];
#pragma unroll
        for (int k = 0; k < R / 2; ++k) {
            e[k] = v[2 * k];
            o[k] = v[2 * k + 1];
        }
        dft<T, R / 2, DIR>(e);
        dft<T, R / 2, DIR>(o);
        static_for<0, R / 2>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            cx<T> t = rot<T, R, k, DIR>(o[k]);
            v[k] = e[k] + t;
            v[k + R / 2] = e[k] - t;
        });
    }
}

// Radix schedule of a length-L FFT: up to three stages.
template <int A, int B = 1, int C = 1>
struct Radices {
    static constexpr int nst = (B == 1) ? 1 : (C == 1 ? 2 : 3);
    static constexpr int L = A * B * C;
    static constexpr int Rmax = (A > B ? (A > C ? A : C) : (B > C ? B : C));
    static constexpr int Tp = L / Rmax;  // threads per pencil
    __host__ __device__ static constexpr int radix(int s) { return s == 0 ? A : s == 1 ? B : C; }
    __host__ __device__ static constexpr int prefix(int s) { return s == 0 ? 1 : s == 1 ? A : A * B; }
    static constexpr int first = A;
    static constexpr int last = (nst == 1) ? A : (nst == 2 ? B : C);
    // the same stages in reverse order: its first radix is this schedule's last
    using Reverse = std::conditional_t<nst == 1, Radices<A>,
                                       std::conditional_t<nst == 2, Radices<B, A>, Radices<C, B, A>>>;
};

// The schedule PL with E >= PL::Rmax elements per thread (E / R butterflies of each stage per
// thread): Tp = L / E threads per pencil.  Fewer threads per pencil for long pencils, so that a
// workgroup of several pencils stays within the register and LDS budget of two workgroups per CU.
template <class PL, int E>
struct Spread : PL {
    static_assert(E % PL::Rmax == 0 && E <= PL::L, "E must be a multiple of the largest radix");
    static constexpr int Rmax = E;
    static constexpr int Tp = PL::L / E;
    using Reverse = Spread<typename PL::Reverse, E>;
};

// Default schedule per length.
template <int L> struct DefaultPlan;
template <> struct DefaultPlan<2> { using type = Radices<2>; };
template <> struct DefaultPlan<4> { using type = Radices<4>; };
template <> struct DefaultPlan<8> { using type = Radices<8>; };
template <> struct DefaultPlan<16> { using type = Radices<4, 4>; };
template <> struct DefaultPlan<32> { using type = Radices<8, 4>; };
template <> struct DefaultPlan<64> { using type = Radices<8, 8>; };
template <> struct DefaultPlan<128> { using type = Radices<8, 16>; };
template <> struct DefaultPlan<256> { using type = Radices<16, 16>; };
template <> struct DefaultPlan<512> { using type = Radices<8, 8, 8>; };
template <> struct DefaultPlan<1024> { using type = Radices<8, 8, 16>; };
template <> struct DefaultPlan<2048> { using type = Radices<8, 16, 16>; };

// Candidate schedules per pass kind and length.  Candidate 0 is the default (measured best on
// MI355X at 512^3 FP32 where the lengths occur there); the autotuner may pick another per plan.
template <class... Ps>
struct PlanList {
    static constexpr int size = sizeof...(Ps);
};
template <int I, class List>
struct ListAt;
template <class P, class... Ps>
struct ListAt<0, PlanList<P, Ps...>> {
    using type = P;
};
template <int I, class P, class... Ps>
struct ListAt<I, PlanList<P, Ps...>> {
    using type = typename ListAt<I - 1, PlanList<Ps...>>::type;
};

// generic candidates: the default schedule and, from 16 up, one alternative split
template <int L> struct AltPlans { using type = PlanList<typename DefaultPlan<L>::type>; };
template <> struct AltPlans<16> { using type = PlanList<Radices<4, 4>, Radices<16>>; };
template <> struct AltPlans<32> { using type = PlanList<Radices<8, 4>, Radices<4, 8>>; };
template <> struct AltPlans<64> { using type = PlanList<Radices<8, 8>, Radices<4, 16>>; };
template <> struct AltPlans<128> { using type = PlanList<Radices<8, 16>, Radices<16, 8>>; };
template <> struct AltPlans<256> { using type = PlanList<Radices<16, 16>, Radices<4, 8, 8>>; };
template <> struct AltPlans<512> { using type = PlanList<Radices<8, 8, 8>, Radices<16, 2, 16>>; };
template <> struct AltPlans<1024> { using type = PlanList<Radices<8, 8, 16>, Radices<16, 4, 16>>; };
template <> struct AltPlans<2048> { using type = PlanList<Radices<8, 16, 16>, Radices<16, 8, 16>>; };

// x forward (r2c, contiguous rows), x inverse (c2r), strided middle axis, last axis
template <int M> struct XFwdCands { using type = typename AltPlans<M>::type; };
template <int M> struct XInvCands { using type = typename AltPlans<M>::type; };
template <> struct XInvCands<256> { using type = PlanList<Radices<8, 4, 8>, Radices<16, 16>>; };
template <int L> struct AxisCands { using type = typename AltPlans<L>::type; };
template <> struct AxisCands<512> { using type = PlanList<Radices<16, 2, 16>, Radices<8, 8, 8>>; };
template <int L> struct LastCands { using type = typename AltPlans<L>::type; };
template <> struct LastCands<512> { using type = PlanList<Radices<2, 16, 16>, Radices<16, 16, 2>>; };

template <int M> struct XFwdPlan { using type = typename ListAt<0, typename XFwdCands<M>::type>::type; };
template <int M> struct XInvPlan { using type = typename ListAt<0, typename XInvCands<M>::type>::type; };
template <int L> struct AxisPlan { using type = typename ListAt<0, typename AxisCands<L>::type>::type; };
template <int L> struct LastPlan { using type = typename ListAt<0, typename LastCands<L>::type>::type; };

// Calls f(PL{}) with the schedule number v of List (v out of range: candidate 0).
template <class List, int I = 0, class F>
__host__ __device__ __forceinline__ auto with_plan(int v, F &&f)
{
    if constexpr (I + 1 >= List::size) {
        return f(typename ListAt<I, List>::type{});
    } else {
        if (v == I) return f(typename ListAt<I, List>::type{});
        return with_plan<List, I + 1>(v, f);
    }
}

// Twiddle W_{Ns R}^{m}, m = (j mod Ns) r, from the table of length Lt (forward sign); conjugated
// for the inverse.
template <typename T, int DIR>
__device__ __forceinline__ cx<T> twiddle(const cx<T> *__restrict__ tw, int lt_shift, int m, int log_nsr)
{
    cx<T> w = tw[m << (lt_shift - log_nsr)];
    return DIR > 0 ? conj(w) : w;
}

__host__ __device__ constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

enum { TW_LT = 0, TW_STAGE = 1 };

// Multiplies v[r], 0 < r < R, by the twiddles W_{Ns R}^{jj r} (conjugated for the inverse).
template <typename T, int R, int Ns, int DIR, int TWM>
__device__ __forceinline__ void apply_twiddles(cx<T> *v, int jj, const cx<T> *__restrict__ tw, int lt_shift)
{
    if constexpr (TWM == TW_STAGE) {
        const cx<T> *st = tw + (1u << lt_shift) + stage_tw_offset(Ns * R, R) + (unsigned)(jj * R);
        if constexpr (sizeof(T) == 4) {
            // FP32: two twiddles per 16-byte load (entry 0 is 1 and is skipped)
            typedef float f32x4 __attribute__((ext_vector_type(4)));
            const f32x4 *q = reinterpret_cast<const f32x4 *>(st);
#pragma unroll
            for (int h = 0; h < R / 2; ++h) {
                const f32x4 w = q[h];
                if (h > 0) v[2 * h] = cmul(v[2 * h], cx<T>{w.x, DIR > 0 ? -w.y : w.y});
                v[2 * h + 1] = cmul(v[2 * h + 1], cx<T>{w.z, DIR > 0 ? -w.w : w.w});
            }
        } else {
#pragma unroll
            for (int r = 1; r < R; ++r) v[r] = cmul(v[r], DIR > 0 ? conj(st[r]) : st[r]);
        }
    } else {
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], twiddle<T, DIR>(tw, lt_shift, jj * r, ilog2c(Ns * R)));
    }
}

// Runs every stage of the schedule PL for one pencil.
// On entry: v[b * R0 + r] = x[t + b Tp + r L / R0] for b < Rmax / R0 (R0 = first radix).
// On exit:  v[b * Rl + r] = X[t + b Tp + r L / Rl] for b < Rmax / Rl (Rl = last radix).
// `lds(e)` returns a reference to this pencil's LDS slot for element e.  Contains workgroup
// barriers, so every thread of the workgroup must call it (idle threads included).  The first LDS
// write is preceded by a barrier, so the caller may have used the same LDS just before.
// G > 1: the workgroup's pencils form G groups (this thread's is `grp`) that take turns in one
// LDS area sized for a single group, so each exchange costs G barrier pairs and 1/G of the LDS.
template <typename T, class PL, int DIR, int TWM = TW_STAGE, int G = 1, class Lds>
__device__ __forceinline__ void fft_stages(cx<T> *v, int t, Lds &&lds, const cx<T> *__restrict__ tw, int lt_shift,
                                           int grp = 0)
{
    constexpr int L = PL::L;
    constexpr int Tp = PL::Tp;
    static_for<0, PL::nst>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        constexpr int R = PL::radix(s);
        constexpr int B = PL::Rmax / R;
        constexpr int Ns = PL::prefix(s);
#pragma unroll
        for (int b = 0; b < B; ++b) dft<T, R, DIR>(&v[b * R]);
        if constexpr (s + 1 < PL::nst) {
            // exchange, then the next stage's inputs and twiddles
            constexpr int R2 = PL::radix(s + 1);
            constexpr int B2 = PL::Rmax / R2;
            constexpr int Ns2 = PL::prefix(s + 1);
#pragma unroll
            for (int gg = 0; gg < G; ++gg) {
                const bool mine = (G == 1) || (grp == gg);
                __syncthreads();
                if (mine) {
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        const int j = t + b * Tp;
                        const int base = (j / Ns) * Ns * R + (j & (Ns - 1));
#pragma unroll
                        for (int r = 0; r < R; ++r) lds(base + r * Ns) = v[b * R + r];
                    }
                }
                __syncthreads();
                if (mine) {
#pragma unroll
                    for (int b = 0; b < B2; ++b) {
                        const int j = t + b * Tp;
#pragma unroll
                        for (int r = 0; r < R2; ++r) v[b * R2 + r] = lds(j + r * (L / R2));
                    }
                }
            }
#pragma unroll
            for (int b = 0; b < B2; ++b)
                apply_twiddles<T, R2, Ns2, DIR, TWM>(&v[b * R2], (t + b * Tp) & (Ns2 - 1), tw, lt_shift);
        }
    });
}

}  // namespace pfc
