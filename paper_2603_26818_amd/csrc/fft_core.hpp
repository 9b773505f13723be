// fft_core.hpp -- device building blocks of the pencil FFTs (gfx950, wave64).
//
// A length-L complex FFT of one "pencil" is done by Tp = L / Rmax threads with a Stockham
// autosort schedule: stage s has radix R_s; each thread runs up to nb(R_s) radix-R_s butterflies from
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

// cos and sin of 2 pi a / b, computed at compile time in long double: the angle is reduced to the
// first octant exactly in integers (units of 2 pi / 8b), then Taylor series (|x| <= pi / 4, 24
// terms: far below long double rounding).  Constants of the in-register DFTs of radices with
// factors 3, 5, 7.
__host__ __device__ constexpr long double taylor_sin(long double x)
{
    long double term = x, sum = x;
    for (int n = 1; n < 24; ++n) {
        term *= -x * x / ((long double)(2 * n) * (long double)(2 * n + 1));
        sum += term;
    }
    return sum;
}
__host__ __device__ constexpr long double taylor_cos(long double x)
{
    long double term = 1.0L, sum = 1.0L;
    for (int n = 1; n < 24; ++n) {
        term *= -x * x / ((long double)(2 * n - 1) * (long double)(2 * n));
        sum += term;
    }
    return sum;
}
// which = 0: cos(2 pi a / b), 1: sin(2 pi a / b)
__host__ __device__ constexpr long double cs2pi(long long a, long long b, int which)
{
    long long u = ((a % b) + b) % b * 8;  // angle = 2 pi u / (8 b), u in [0, 8b)
    long double sc = 1.0L, ss = 1.0L;
    bool swap = false;
    if (u > 4 * b) {  // (pi, 2 pi): reflect, sin changes sign
        u = 8 * b - u;
        ss = -ss;
    }
    if (u > 2 * b) {  // (pi/2, pi]: cos changes sign
        u = 4 * b - u;
        sc = -sc;
    }
    if (u > b) {  // (pi/4, pi/2]: cos and sin exchange
        u = 2 * b - u;
        swap = true;
    }
    const long double x = 6.283185307179586476925286766559005768L * (long double)u / (long double)(8 * b);
    const long double c = swap ? taylor_sin(x) : taylor_cos(x), sn = swap ? taylor_cos(x) : taylor_sin(x);
    return which == 0 ? sc * c : ss * sn;
}

__host__ __device__ constexpr bool is_pow2c(int v) { return v > 0 && (v & (v - 1)) == 0; }
__host__ __device__ constexpr int smallest_factor(int v)
{
    for (int f = 2; f * f <= v; ++f)
        if (v % f == 0) return f;
    return v;
}
__host__ __device__ constexpr int gcdc(int a, int b) { return b == 0 ? a : gcdc(b, a % b); }
__host__ __device__ constexpr int lcmc(int a, int b) { return a / gcdc(a, b) * b; }

// a * exp(DIR * 2 pi i K / R) for any R (exact for multiples of a quarter turn).
template <typename T, int R, int K, int DIR>
__device__ __forceinline__ cx<T> rotg(cx<T> a)
{
    constexpr int k = ((K % R) + R) % R;
    if constexpr (16 % R == 0) {
        return rot<T, R, k, DIR>(a);
    } else if constexpr (k == 0) {
        return a;
    } else if constexpr (2 * k == R) {
        return {-a.x, -a.y};
    } else if constexpr (4 * k == R) {
        return DIR > 0 ? mul_i(a) : mul_mi(a);
    } else if constexpr (4 * k == 3 * R) {
        return DIR > 0 ? mul_mi(a) : mul_i(a);
    } else {
        constexpr T c = (T)cs2pi(k, R, 0);
        constexpr T sn = (T)(DIR * cs2pi(k, R, 1));
        return {a.x * c - a.y * sn, a.x * sn + a.y * c};
    }
}

// In-register DFT of size R, natural order in and out, fully unrolled.  Powers of two: radix-2
// decimation in time.  Other R (factors 2, 3, 5, 7): decimation in time over the smallest prime
// factor p (q = R / p): X[k + q s] = sum_r W_p^{r s} W_R^{r k} DFT_q(v[r], v[r + p], ...)[k]; a
// prime R is summed directly.
template <typename T, int R, int DIR>
__device__ __forceinline__ void dft(cx<T> *v)
{
    if constexpr (!is_pow2c(R)) {
        constexpr int p = smallest_factor(R), q = R / p;
        if constexpr (q == 1) {
            // prime R: pair x_r with x_{R-r}, a_r = x_r + x_{R-r}, b_r = x_r - x_{R-r} (r <= H);
            // with c = cos(2 pi r s / R), sn = sin(2 pi r s / R):
            //   X_s = x_0 + sum_r c a_r + DIR i sum_r sn b_r,  X_{R-s} = the same with -DIR i
            // (real-times-complex products: a quarter of the multiplications of the direct sum)
            constexpr int H = (R - 1) / 2;
            cx<T> a[H + 1], b[H + 1];
            cx<T> sum = v[0];
#pragma unroll
            for (int r = 1; r <= H; ++r) {
                a[r] = v[r] + v[R - r];
                b[r] = v[r] - v[R - r];
                sum = sum + a[r];
            }
            const cx<T> x0 = v[0];
            static_for<1, H + 1>([&](auto sc) {
                constexpr int s2 = decltype(sc)::value;
                cx<T> A = x0, Bv = {T(0), T(0)};
                static_for<1, H + 1>([&](auto rc) {
                    constexpr int r = decltype(rc)::value;
                    constexpr T c = (T)cs2pi(r * s2, R, 0), sn = (T)cs2pi(r * s2, R, 1);
                    A = {A.x + c * a[r].x, A.y + c * a[r].y};
                    Bv = {Bv.x + sn * b[r].x, Bv.y + sn * b[r].y};
                });
                // DIR i B = DIR (-B.y, B.x)
                const cx<T> iB = {T(-DIR) * Bv.y, T(DIR) * Bv.x};
                v[s2] = A + iB;
                v[R - s2] = A - iB;
            });
            v[0] = sum;
        } else {
            cx<T> e[p][q];
#pragma unroll
            for (int r = 0; r < p; ++r) {
#pragma unroll
                for (int j = 0; j < q; ++j) e[r][j] = v[r + p * j];
                dft<T, q, DIR>(e[r]);
            }
            static_for<0, q>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                cx<T> tt[p];
                static_for<0, p>([&](auto rc) {
                    constexpr int r = decltype(rc)::value;
                    tt[r] = rotg<T, R, r * k, DIR>(e[r][k]);
                });
                static_for<0, p>([&](auto sc) {
                    constexpr int s2 = decltype(sc)::value;
                    cx<T> acc = tt[0];
                    static_for<1, p>([&](auto rc) {
                        constexpr int r = decltype(rc)::value;
                        acc = acc + rotg<T, p, r * s2, DIR>(tt[r]);
                    });
                    v[k + q * s2] = acc;
                });
            });
        }
    } else if constexpr (R == 2) {
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

// Radix schedule of a length-L FFT: up to three stages, Tp threads per pencil.  Stage s has L / R_s
// butterflies; thread t runs butterflies j = t + b Tp, b < nb(R_s) = ceil(L / R_s / Tp), those with
// j < L / R_s ("ragged" stages when Tp does not divide L / R_s).  TP = 0: Tp = L / lcm of the
// radices, so that every stage divides evenly (the largest radix for powers of two).  Rmax: the
// elements a thread holds, max over stages of nb(R) R.
template <int A, int B = 1, int C = 1, int TP = 0>
struct Radices {
    static constexpr int nst = (B == 1) ? 1 : (C == 1 ? 2 : 3);
    static constexpr int L = A * B * C;
    static constexpr int Tp = TP > 0 ? TP : L / lcmc(lcmc(A, B), C);  // threads per pencil
    __host__ __device__ static constexpr int nb(int R) { return (L / R + Tp - 1) / Tp; }
    __host__ __device__ static constexpr bool even(int R) { return (L / R) % Tp == 0; }
    // butterfly j of a radix-R stage exists
    __host__ __device__ static constexpr bool jok(int j, int R) { return even(R) || j < L / R; }
    static constexpr int Rmax = (nb(A) * A > nb(B) * B ? (nb(A) * A > nb(C) * C ? nb(A) * A : nb(C) * C)
                                                       : (nb(B) * B > nb(C) * C ? nb(B) * B : nb(C) * C));
    __host__ __device__ static constexpr int radix(int s) { return s == 0 ? A : s == 1 ? B : C; }
    __host__ __device__ static constexpr int prefix(int s) { return s == 0 ? 1 : s == 1 ? A : A * B; }
    static constexpr int first = A;
    static constexpr int last = (nst == 1) ? A : (nst == 2 ? B : C);
    // the same stages in reverse order: its first radix is this schedule's last
    using Reverse = std::conditional_t<nst == 1, Radices<A, 1, 1, TP>,
                                       std::conditional_t<nst == 2, Radices<B, A, 1, TP>, Radices<C, B, A, TP>>>;
};

// Offset of stage s in a table of per-stage blocks (prefix(s) * radix(s) entries each).
template <class P>
__host__ __device__ constexpr int stage_blocks_off(int s)
{
    int o = 0;
    for (int i = 0; i < s; ++i) o += P::prefix(i) * P::radix(i);
    return o;
}
template <class P, class Q>
__host__ __device__ constexpr bool same_stages()
{
    if (P::nst != Q::nst) return false;
    for (int i = 0; i < P::nst; ++i)
        if (P::radix(i) != Q::radix(i)) return false;
    return true;
}

// The schedule PL with E >= PL::Rmax elements per thread (E / R butterflies of each stage per
// thread): Tp = L / E threads per pencil.  Fewer threads per pencil for long pencils, so that a
// workgroup of several pencils stays within the register and LDS budget of two workgroups per CU.
template <class PL, int E>
struct Spread : PL {
    static_assert(E % PL::Rmax == 0 && E <= PL::L && PL::even(PL::first), "E must be a multiple of every radix");
    static constexpr int Rmax = E;
    static constexpr int Tp = PL::L / E;
    __host__ __device__ static constexpr int nb(int R) { return E / R; }
    __host__ __device__ static constexpr bool even(int) { return true; }
    __host__ __device__ static constexpr bool jok(int, int) { return true; }
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
// lengths with factors 3, 5, 7 (one schedule each; elements per thread = lcm of the radices)
template <> struct DefaultPlan<6> { using type = Radices<6>; };
template <> struct DefaultPlan<10> { using type = Radices<10>; };
template <> struct DefaultPlan<12> { using type = Radices<12>; };
template <> struct DefaultPlan<14> { using type = Radices<14>; };
template <> struct DefaultPlan<15> { using type = Radices<15>; };
template <> struct DefaultPlan<20> { using type = Radices<10, 2>; };
template <> struct DefaultPlan<30> { using type = Radices<10, 3>; };
template <> struct DefaultPlan<60> { using type = Radices<10, 6>; };
template <> struct DefaultPlan<150> { using type = Radices<10, 15>; };
template <> struct DefaultPlan<375> { using type = Radices<15, 5, 5>; };
template <> struct DefaultPlan<750> { using type = Radices<15, 10, 5>; };
// 700 = 7 10 10 and 1400 = 14 10 10 have lcm 70: 50 threads per pencil with ragged stages instead
template <> struct DefaultPlan<700> { using type = Radices<7, 10, 10, 50>; };
template <> struct DefaultPlan<1400> { using type = Radices<14, 10, 10, 50>; };
// the schedule whose twiddle table a non-power-of-two length carries
template <int L>
struct MixPlan {
    using type = typename DefaultPlan<L>::type;
};
template <int L>
struct MixTable {
    using F = typename MixPlan<L>::type;
    using Rv = typename F::Reverse;
    static constexpr int split = stage_blocks_off<F>(F::nst) + stage_blocks_off<Rv>(Rv::nst);
    static constexpr int size = split + L;  // entries, with the x-pass split twiddles
};

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

// A candidate of a strided pass that brings its own tile instead of the length's default
// (PencilTile in kernels.hpp): SEGB bytes of adjacent columns per workgroup (the row segment each
// load and store instruction moves), E elements per thread (0: the schedule's own), G LDS groups,
// PF state prefetch in the step.  PL is the radix schedule.
template <class PL, int SEGB, int E = 0, int G = 1, bool PF = true>
struct Tiled {
    using plan = PL;
    static constexpr int L = PL::L, seg_bytes = SEGB, elems = E, groups = G;
    static constexpr bool prefetch = PF;
};

// x forward (r2c, contiguous rows), x inverse (c2r), strided middle axis, last axis
template <int M> struct XFwdCands { using type = typename AltPlans<M>::type; };
template <int M> struct XInvCands { using type = typename AltPlans<M>::type; };
template <> struct XInvCands<256> { using type = PlanList<Radices<8, 4, 8>, Radices<16, 16>>; };
// x rows of 375 and 700 points (the x passes of the 750^3 and 1400^3 grids): the radices ragged
// over 32 or 64 threads, so that every row starts at a half or a whole wavefront, then the lcm or
// 50-thread schedules.  Measured at 750^3 FP32: x r2c 0.99 against 1.29 ms, x c2r 1.06 against
// 1.15 ms; at 1400^3: 6.77 against 6.88 ms and 8.15 against 8.36 ms.
template <> struct XFwdCands<375> { using type = PlanList<Radices<15, 5, 5, 32>, Radices<15, 5, 5>>; };
template <> struct XInvCands<375> { using type = PlanList<Radices<15, 5, 5, 32>, Radices<15, 5, 5>>; };
template <> struct XFwdCands<700> { using type = PlanList<Radices<7, 10, 10, 64>, Radices<7, 10, 10, 50>>; };
template <> struct XInvCands<700> { using type = PlanList<Radices<7, 10, 10, 64>, Radices<7, 10, 10, 50>>; };
// x rows of 1024 points (x = 2048): 16 4 16 first, measured at 2048^3 FP32: x r2c 15.1 against
// 15.6 ms, x c2r 18.0 against 20.2 ms
template <> struct XFwdCands<1024> { using type = PlanList<Radices<16, 4, 16>, Radices<8, 8, 16>>; };
template <> struct XInvCands<1024> { using type = PlanList<Radices<16, 4, 16>, Radices<8, 8, 16>>; };
template <int L> struct AxisCands { using type = typename AltPlans<L>::type; };
template <> struct AxisCands<512> {
    using type = PlanList<Radices<16, 2, 16>, Radices<8, 8, 8>, Tiled<Radices<16, 2, 16>, 256>,
                          Tiled<Radices<16, 2, 16>, 256, 32, 2>>;
};
template <int L> struct LastCands { using type = typename AltPlans<L>::type; };
template <> struct LastCands<512> { using type = PlanList<Radices<2, 16, 16>, Radices<16, 16, 2>>; };
// the last axis of a 3D step (z): the 2D list, and at 512 tiles of 256-byte row segments (the
// pencils' elements lie a whole z plane apart, so each element row of a tile is one segment)
template <int L> struct ZCands { using type = typename LastCands<L>::type; };
// 750 (z, y and the other last-axis passes): 15 10 5 (every element step even, so that the
// last-axis passes can address blocks of plane pairs), ragged over 50 threads per pencil (at most
// 20 elements each: 800 threads in one workgroup per CU, which its 96 KB of LDS allows), and the
// lcm schedule (25 threads of 30 elements: 400 threads).  Measured at 750^3 FP32 with 10 15 5: z
// 2.20 against 2.86 ms.  Narrower z tiles, so that two workgroups share a CU, measured slower: half
// a line (8 pencils, 48 KB) 2.23 ms, two LDS groups (48 KB) 2.43 ms; so did persistent workgroups
// looping over the tiles at 512^3 (z 539 against 506 us).
template <> struct ZCands<750> { using type = PlanList<Radices<15, 10, 5, 50>, Radices<15, 10, 5>>; };
template <> struct LastCands<750> { using type = PlanList<Radices<15, 10, 5, 50>>; };
// y at 750: half-line tiles (8 pencils, 48 KB, two workgroups per CU; the plane order keeps the two
// tiles of a line on one XCD) first: 0.74 against 0.85 ms per direction at 750^3 FP32
template <> struct AxisCands<750> {
    using type = PlanList<Tiled<Radices<15, 10, 5, 50>, 64, 0, 1, false>, Radices<15, 10, 5, 50>, Radices<15, 10, 5>>;
};
// 2048-point y and z pencils (2048^3): 16 8 16 first, measured at 2048^3 FP32: y 16.2 against
// 16.5 ms per direction, z 39.4 against 40.0 ms
template <> struct ZCands<2048> { using type = PlanList<Radices<16, 8, 16>, Radices<8, 16, 16>>; };
template <> struct AxisCands<2048> { using type = PlanList<Radices<16, 8, 16>, Radices<8, 16, 16>>; };
template <> struct ZCands<512> {
    using type = PlanList<Radices<2, 16, 16>, Radices<16, 16, 2>, Tiled<Radices<2, 16, 16>, 256>,
                          Tiled<Radices<2, 16, 16>, 256, 32, 2, false>, Tiled<Radices<2, 16, 16>, 256, 32, 1, false>>;
};
// The z candidates per dtype: the same list, except FP32 at 512, which takes 16 16 2 first (with
// the plane-pair layout, 512^3: z 491 against 499 us; FP64 keeps 2 16 16: 865 against 871 us).
template <typename T, int L> struct ZCandsOf { using type = typename ZCands<L>::type; };
template <> struct ZCandsOf<float, 512> {
    using type = PlanList<Radices<16, 16, 2>, Radices<2, 16, 16>, Tiled<Radices<2, 16, 16>, 256>,
                          Tiled<Radices<2, 16, 16>, 256, 32, 2, false>, Tiled<Radices<2, 16, 16>, 256, 32, 1, false>>;
};
static_assert(ZCandsOf<float, 512>::type::size == ZCands<512>::type::size, "one candidate count per length");

// The radix schedule of a candidate (a Tiled candidate's own; the default candidate's schedule is
// what the other kernels of a length take, with the length's default tile)
template <class C, class = void>
struct PlanOf {
    using type = C;
};
template <class C>
struct PlanOf<C, std::void_t<typename C::plan>> {
    using type = typename C::plan;
};
template <int M> struct XFwdPlan { using type = typename PlanOf<typename ListAt<0, typename XFwdCands<M>::type>::type>::type; };
template <int M> struct XInvPlan { using type = typename PlanOf<typename ListAt<0, typename XInvCands<M>::type>::type>::type; };
template <int L> struct AxisPlan { using type = typename PlanOf<typename ListAt<0, typename AxisCands<L>::type>::type>::type; };
template <int L> struct LastPlan { using type = typename PlanOf<typename ListAt<0, typename LastCands<L>::type>::type>::type; };

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

enum { TW_LT = 0, TW_STAGE = 1, TW_MIX = 2 };

// Twiddle table of a length L that is not a power of two (TW_MIX; one table per such length of a
// plan, at the pointer the kernel receives): for the length's schedule F and then for F's reverse,
// per stage s a block of prefix(s) * radix(s) entries, entry jj R + r = W_{Ns R}^{jj r}; then the
// x-pass split twiddles W_{2L}^k, k < L.
// Multiplies v[r], 0 < r < R, by the twiddles W_{Ns R}^{jj r} of stage s of schedule PL
// (conjugated for the inverse).
template <typename T, class PL, int s, int DIR, int TWM>
__device__ __forceinline__ void apply_twiddles(cx<T> *v, int jj, const cx<T> *__restrict__ tw, int lt_shift)
{
    constexpr int R = PL::radix(s), Ns = PL::prefix(s);
    if constexpr (TWM == TW_MIX) {
        using F = typename MixPlan<PL::L>::type;
        static_assert(same_stages<PL, F>() || same_stages<PL, typename F::Reverse>(),
                      "a schedule of a length that is not a power of two takes the stages of its table");
        constexpr int base = same_stages<PL, F>() ? 0 : stage_blocks_off<F>(F::nst);
        const cx<T> *st = tw + base + stage_blocks_off<PL>(s) + (unsigned)(jj * R);
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], DIR > 0 ? conj(st[r]) : st[r]);
    } else if constexpr (TWM == TW_STAGE) {
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
// On entry: v[b * R0 + r] = x[t + b Tp + r L / R0] for b < nb(R0) (R0 = first radix), where that
// butterfly exists (jok).  On exit: v[b * Rl + r] = X[t + b Tp + r L / Rl] for b < nb(Rl) likewise
// (Rl = last radix).
// `lds(e)` returns a reference to this pencil's LDS slot for element e.  Contains workgroup
// barriers, so every thread of the workgroup must call it (idle threads included).  The first LDS
// write is preceded by a barrier, so the caller may have used the same LDS just before.
// G > 1: the workgroup's pencils form G groups (this thread's is `grp`) that take turns in one
// LDS area sized for a single group, so each exchange costs G barrier pairs and 1/G of the LDS.
// Lengths that are not powers of two always take their own table (TW_MIX).
template <typename T, class PL, int DIR, int TWM = TW_STAGE, int G = 1, class Lds>
__device__ __forceinline__ void fft_stages(cx<T> *v, int t, Lds &&lds, const cx<T> *__restrict__ tw, int lt_shift,
                                           int grp = 0)
{
    constexpr int L = PL::L;
    constexpr int Tp = PL::Tp;
    constexpr int TW = is_pow2c(L) ? TWM : TW_MIX;
    static_for<0, PL::nst>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        constexpr int R = PL::radix(s);
        constexpr int B = PL::nb(R);
        constexpr int Ns = PL::prefix(s);
#pragma unroll
        for (int b = 0; b < B; ++b) dft<T, R, DIR>(&v[b * R]);  // (absent butterflies: unused values)
        if constexpr (s + 1 < PL::nst) {
            // exchange, then the next stage's inputs and twiddles
            constexpr int R2 = PL::radix(s + 1);
            constexpr int B2 = PL::nb(R2);
            constexpr unsigned Ns2 = PL::prefix(s + 1);
#pragma unroll
            for (int gg = 0; gg < G; ++gg) {
                const bool mine = (G == 1) || (grp == gg);
                __syncthreads();
                if (mine) {
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        const unsigned j = t + b * Tp;
                        const int base = (int)((j / Ns) * Ns * R + j % Ns);
                        if (PL::jok(j, R)) {
#pragma unroll
                            for (int r = 0; r < R; ++r) lds(base + r * Ns) = v[b * R + r];
                        }
                    }
                }
                __syncthreads();
                if (mine) {
#pragma unroll
                    for (int b = 0; b < B2; ++b) {
                        const int j = t + b * Tp;
                        if (PL::jok(j, R2)) {
#pragma unroll
                            for (int r = 0; r < R2; ++r) v[b * R2 + r] = lds(j + r * (L / R2));
                        }
                    }
                }
            }
#pragma unroll
            for (int b = 0; b < B2; ++b)
                apply_twiddles<T, PL, s + 1, DIR, TW>(&v[b * R2], (int)((unsigned)(t + b * Tp) % Ns2), tw, lt_shift);
        }
    });
}

}  // namespace pfc
