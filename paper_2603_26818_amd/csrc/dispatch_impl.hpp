// dispatch_impl.hpp -- length dispatch of the kernel templates; included once per dtype.
#pragma once

#include "kernels.hpp"
#include "launch.hpp"

namespace pfc {

template <class F>
static hipError_t by_length(int64_t L, F &&f)
{
    switch (L) {
    case 2: return f(std::integral_constant<int, 2>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 8: return f(std::integral_constant<int, 8>{});
    case 16: return f(std::integral_constant<int, 16>{});
    case 32: return f(std::integral_constant<int, 32>{});
    case 64: return f(std::integral_constant<int, 64>{});
    case 128: return f(std::integral_constant<int, 128>{});
    case 256: return f(std::integral_constant<int, 256>{});
    case 512: return f(std::integral_constant<int, 512>{});
    case 1024: return f(std::integral_constant<int, 1024>{});
    case 2048: return f(std::integral_constant<int, 2048>{});
    case 6: return f(std::integral_constant<int, 6>{});
    case 10: return f(std::integral_constant<int, 10>{});
    case 12: return f(std::integral_constant<int, 12>{});
    case 14: return f(std::integral_constant<int, 14>{});
    case 15: return f(std::integral_constant<int, 15>{});
    case 20: return f(std::integral_constant<int, 20>{});
    case 30: return f(std::integral_constant<int, 30>{});
    case 60: return f(std::integral_constant<int, 60>{});
    case 150: return f(std::integral_constant<int, 150>{});
    case 375: return f(std::integral_constant<int, 375>{});
    case 700: return f(std::integral_constant<int, 700>{});
    case 750: return f(std::integral_constant<int, 750>{});
    case 1400: return f(std::integral_constant<int, 1400>{});
    default: return hipErrorInvalidValue;
    }
}

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Calls f(std::bool_constant<nt>).
template <class F>
static hipError_t with_nt(bool nt, F &&f)
{
    return nt ? f(std::true_type{}) : f(std::false_type{});
}

// Every element step of the schedule PL (b Tp + r L / R for its first and last radix) is a
// multiple of the layout's plane block 2^zs, as the last-axis addressing requires (AxisMap, Pack).
template <class PL>
static bool z_steps_ok(int zs)
{
    const int Z = 1 << zs;
    return PL::Tp % Z == 0 && (PL::L / PL::first) % Z == 0 && (PL::L / PL::last) % Z == 0;
}

// Whether blocks of 2^zs z planes suit this geometry's last-axis passes: the step's default z
// schedule and the schedule of the other last-axis passes (state set-up, export, transforms) step
// by multiples of the block.
template <typename T>
bool z_blocks_ok(const Geom &g, int zs)
{
    bool ok = false;
    (void)by_length(g.n0, [&](auto Lc) -> hipError_t {
        constexpr int L = decltype(Lc)::value;
        using TO = TileOf<T, typename ListAt<0, typename ZCandsOf<T, L>::type>::type>;
        using PZ = SpreadIf<typename TO::plan, TO::tile::E>;
        using P0 = SpreadIf<typename LastPlan<L>::type, PencilTile<T, L>::E>;
        ok = z_steps_ok<PZ>(zs) && z_steps_ok<P0>(zs) && z_steps_ok<typename LastPlan<L>::type>(zs);
        return hipSuccess;
    });
    return ok;
}

// Addressing of the middle-axis (3D y) pass: batch = z plane, columns kx, elements y.
static inline AxisMap y_map(const Geom &g)
{
    const Pack pk = pack_of(g);
    return AxisMap{pk.nrows * pk.Mp << pk.zs, pk.Mp << pk.zs, 0, 0, pk.zs, 0, pk.zs, pk.cs};
}
// Addressing of a last-axis c2c pass: one batch, columns row M + kx, elements along the last axis.
static inline AxisMap last_map(const Geom &g)
{
    const Pack pk = pack_of(g);
    return AxisMap{0, pk.e_stride(), pk.Mp << pk.zs, g.M, 0, pk.zs, pk.zs, pk.cs};
}

// Largest even width <= w (w >= 2).
static inline int even_width(int w) { return w > 1 ? (w & ~1) : w; }

// Workgroups per 128-byte line for column tiles of W complex values (1 for whole-line tiles).
template <typename T>
static int line_group(int W)
{
    const int bytes = W * (int)sizeof(cx<T>);
    return bytes >= 128 ? 1 : 128 / bytes;
}

// Rows per workgroup of the x inverse pass: one wavefront (measured faster than 256 threads; the
// pass's LDS round trips then need no cross-wave barrier), except for mixed-radix rows that fill
// most of a wavefront without dividing it (700 points over 50 threads), which take about 256
// threads as the forward pass does (1400^3 FP32: 8.3 against 9.0 ms).  Over 64 threads a 700-point
// row is one whole wavefront: 7.1 against 8.0 ms with four rows per workgroup; 375-point rows take
// two per wavefront (256 threads measured slower: 1.23 against 1.14 ms).
template <class PL>
struct XInvRows {
    static constexpr int value = (!is_pow2c(PL::L) && PL::Tp > 32 && PL::Tp < 64) ? XRows<PL>::value
                                                                                   : ((64 / PL::Tp) < 1 ? 1 : 64 / PL::Tp);
};

template <typename T>
hipError_t launch_x_r2c(const Geom &g, const T *in, cx<T> *out, bool cube, const cx<T> *tw, hipStream_t s,
                        int variant)
{
    if (!layout_ok(g)) return hipErrorInvalidValue;
    return by_length(g.M, [&](auto Mc) -> hipError_t {
        constexpr int M = decltype(Mc)::value;
        if constexpr (M > 1024) {
            return hipErrorInvalidValue;
        } else {
            auto run = [&](auto plc, auto cubec) -> hipError_t {
                using PL = decltype(plc);
                constexpr bool CUBE = decltype(cubec)::value;
                constexpr int ROWS = XRows<PL>::value;
                const dim3 grid((unsigned)cdiv(g.xrows, ROWS)), block(ROWS * PL::Tp);
                // non-temporal hints measured faster at M = 256 and slower at M = 1024; mixed-radix
                // rows are not whole lines (their partial lines then reach HBM unmerged).  Padded
                // LDS rows (power-of-two M): 512^3 FP64 x r2c 0.360 against 0.389 ms, FP32 even.
                return with_nt(g.nt && M < 1024 && is_pow2c(M), [&](auto ntc) -> hipError_t {
                    hipLaunchKernelGGL((x_r2c_kernel<T, PL, ROWS, CUBE, is_pow2c(M), decltype(ntc)::value>), grid, block, 0,
                                       s, in, out, g.xrows, tw + g.tw_x, g.lt_shift, pack_of(g));
                    return hipGetLastError();
                });
            };
            if (!cube) return run(typename XFwdPlan<M>::type{}, std::false_type{});
            return with_plan<typename XFwdCands<M>::type>(variant, [&](auto plc) { return run(plc, std::true_type{}); });
        }
    });
}

template <typename T>
hipError_t launch_x_c2r(const Geom &g, const cx<T> *in, T *out, const cx<T> *tw, hipStream_t s, int variant)
{
    if (!layout_ok(g)) return hipErrorInvalidValue;
    return by_length(g.M, [&](auto Mc) -> hipError_t {
        constexpr int M = decltype(Mc)::value;
        if constexpr (M > 1024) {
            return hipErrorInvalidValue;
        } else {
            return with_plan<typename XInvCands<M>::type>(variant, [&](auto plc) -> hipError_t {
                using PL = decltype(plc);
                constexpr int ROWS = XInvRows<PL>::value;
                const dim3 grid((unsigned)cdiv(g.xrows, ROWS)), block(ROWS * PL::Tp);
                const T sc = (T)(1.0 / ((double)g.M * (double)g.n0 * (double)g.nrows));
                AdjEpi<T> ea{};
                // unpadded LDS rows: padded ones measured slower here (512^3 FP32 0.224 against
                // 0.215 ms, FP64 0.419 against 0.396 ms, 2048^3 FP32 18.5 against 18.0 ms)
                return with_nt(g.nt && is_pow2c(M), [&](auto ntc) -> hipError_t {
                    hipLaunchKernelGGL((x_c2r_kernel<T, PL, ROWS, EPI_PLAIN, false, false, decltype(ntc)::value>), grid,
                                       block, 0, s, in, out, g.xrows, tw + g.tw_x, g.lt_shift, sc, ea, pack_of(g));
                    return hipGetLastError();
                });
            });
        }
    });
}

// The fused x pass between two steps of the single-plan step (x c2r of one step, the cube, x r2c of
// the next; x_c2r_r2c_kernel), in place on the packed spectrum, on the default x schedules of both
// directions, one wavefront per workgroup.  A geometry has it when both schedules' threads per row
// divide a wavefront and the rows are shorter than 1024 points.  The arithmetic is that of the two
// separate passes, bit for bit.  Measured against the separate passes (whole steps): 512^3 FP32
// 825 against 781 steps/s, FP64 429 against 415, 750^3 186 against 183; at 2048^3 (1024-point rows,
// one row per workgroup) 108.4 against 104.6 ms per step, so rows of 1024 keep the separate passes.
template <class PLI, class PLF>
struct XStepFused {
    static constexpr bool ok = PLI::L == PLF::L && PLI::L < 1024 && PLI::Tp <= 64 && PLF::Tp <= 64 &&
                               64 % PLI::Tp == 0 && 64 % PLF::Tp == 0 && XFused<PLI, PLF, 64>::ok;
};

template <typename T>
bool x_fused_ok(const Geom &g)
{
    if (!layout_ok(g)) return false;
    bool ok = false;
    (void)by_length(g.M, [&](auto Mc) -> hipError_t {
        constexpr int M = decltype(Mc)::value;
        if constexpr (M <= 1024) ok = XStepFused<typename XInvPlan<M>::type, typename XFwdPlan<M>::type>::ok;
        return hipSuccess;
    });
    return ok;
}

template <typename T>
hipError_t launch_x_c2r_r2c(const Geom &g, cx<T> *data, const cx<T> *tw, hipStream_t s)
{
    if (!layout_ok(g)) return hipErrorInvalidValue;
    return by_length(g.M, [&](auto Mc) -> hipError_t {
        constexpr int M = decltype(Mc)::value;
        if constexpr (M > 1024) {
            return hipErrorInvalidValue;
        } else {
            using PLI = typename XInvPlan<M>::type;
            using PLF = typename XFwdPlan<M>::type;
            if constexpr (!XStepFused<PLI, PLF>::ok) {
                return hipErrorInvalidValue;
            } else {
                constexpr int R = XFused<PLI, PLF, 64>::R;
                const dim3 grid((unsigned)cdiv(g.xrows, R)), block(64);
                const T sc = (T)(1.0 / ((double)g.M * (double)g.n0 * (double)g.nrows));
                // ordinary loads and stores: non-temporal hints (as the separate x passes take them)
                // measured 1.3 % slower per 512^3 FP32 step, the same in FP64.  Padded LDS rows
                // (power-of-two M): FP64 steps 438 against 431 steps/s at 512^3, 2768 against 2671
                // at 256^3; FP32 even.
                hipLaunchKernelGGL((x_c2r_r2c_kernel<T, PLI, PLF, 64, false, is_pow2c(M)>), grid, block, 0, s, data, g.xrows,
                                   tw + g.tw_x, g.lt_shift, sc, pack_of(g));
                return hipGetLastError();
            }
        }
    });
}

template <typename T>
hipError_t launch_x_c2r_adjoint(const Geom &g, const cx<T> *mu, const cx<T> *nu, const T *psi_n, const T *psi_np1,
                                T *out, T c3, double *partial, int64_t *nblocks, const cx<T> *tw, hipStream_t s)
{
    if (!layout_ok(g)) return hipErrorInvalidValue;
    return by_length(g.M, [&](auto Mc) -> hipError_t {
        constexpr int M = decltype(Mc)::value;
        if constexpr (M > 1024) {
            return hipErrorInvalidValue;
        } else {
            using PL = typename XInvPlan<M>::type;
            constexpr int ROWS = XRows<PL>::value;
            const int64_t nb = cdiv(g.xrows, ROWS);
            *nblocks = nb;
            const dim3 grid((unsigned)nb), block(ROWS * PL::Tp);
            const T sc = (T)(1.0 / ((double)g.M * (double)g.n0 * (double)g.nrows));
            AdjEpi<T> ea{nu, psi_n, psi_np1, c3, partial};
            hipLaunchKernelGGL((x_c2r_kernel<T, PL, ROWS, EPI_ADJOINT>), grid, block, 0, s, mu, out, g.xrows,
                               tw + g.tw_x, g.lt_shift, sc, ea, pack_of(g));
            return hipGetLastError();
        }
    });
}

template <typename T>
hipError_t launch_x_c2r_mac(const Geom &g, const cx<T> *in, T *out, const T *w, bool add, const cx<T> *tw,
                            hipStream_t s)
{
    if (!layout_ok(g)) return hipErrorInvalidValue;
    return by_length(g.M, [&](auto Mc) -> hipError_t {
        constexpr int M = decltype(Mc)::value;
        if constexpr (M > 1024) {
            return hipErrorInvalidValue;
        } else {
            using PL = typename XInvPlan<M>::type;
            constexpr int ROWS = XInvRows<PL>::value;
            const dim3 grid((unsigned)cdiv(g.xrows, ROWS)), block(ROWS * PL::Tp);
            const T sc = (T)(1.0 / ((double)g.M * (double)g.n0 * (double)g.nrows));
            AdjEpi<T> ea{};
            ea.w = w;
            ea.add = add ? 1 : 0;
            hipLaunchKernelGGL((x_c2r_kernel<T, PL, ROWS, EPI_MAC>), grid, block, 0, s, in, out, g.xrows, tw + g.tw_x,
                               g.lt_shift, sc, ea, pack_of(g));
            return hipGetLastError();
        }
    });
}

template <typename T>
hipError_t launch_spec_update(const Geom &g, int op, cx<T> *out, const cx<T> *x0, const cx<T> *x1,
                              const HydroArgs &h, hipStream_t s)
{
    if (!layout_ok(g)) return hipErrorInvalidValue;
    static_assert(HYDRO_PSI == HY_PSI && HYDRO_MU == HY_MU && HYDRO_VEL == HY_VEL, "mode codes");
    const int64_t n = g.n0 * g.nrows * g.M;
    const dim3 grid((unsigned)(cdiv(n, 256) < 16384 ? cdiv(n, 256) : 16384)), block(256);
    switch (op) {
    case HY_PSI:
        hipLaunchKernelGGL((spec_update_kernel<T, HY_PSI>), grid, block, 0, s, out, x0, x1, g.n0, g.nrows, g.M, h,
                           pack_of(g));
        break;
    case HY_MU:
        hipLaunchKernelGGL((spec_update_kernel<T, HY_MU>), grid, block, 0, s, out, x0, x1, g.n0, g.nrows, g.M, h,
                           pack_of(g));
        break;
    case HY_VEL:
        hipLaunchKernelGGL((spec_update_kernel<T, HY_VEL>), grid, block, 0, s, out, x0, x1, g.n0, g.nrows, g.M, h,
                           pack_of(g));
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_y_c2c(const Geom &g, cx<T> *data, int dir, const cx<T> *tw, hipStream_t s, int variant)
{
    if (!layout_ok(g)) return hipErrorInvalidValue;
    return by_length(g.n1, [&](auto Lc) -> hipError_t {
        constexpr int L = decltype(Lc)::value;
        if constexpr (L < 4) {
            return hipErrorInvalidValue;
        } else {
            return with_plan<typename AxisCands<L>::type>(variant, [&](auto plc) -> hipError_t {
                using TO = TileOf<T, decltype(plc)>;
                using TL = typename TO::tile;
                using PL = SpreadIf<typename TO::plan, TL::E>;
                constexpr int WM = TL::W;
                const int W = (int)(g.M < WM ? g.M : WM);
                const int64_t tiles = cdiv(g.M, W);
                const dim3 grid((unsigned)(tiles * g.n0)), block(WM * PL::Tp);
                // whole-line tiles: whole planes per XCD (xg = 0, see axis_c2c_kernel), except the
                // grouped power-of-two tiles (2048 points), where it measured slower
                const int xg = (line_group<T>(W) == 1 && (TL::G == 1 || !is_pow2c(L))) ? 0 : line_group<T>(W);
                // non-temporal only with whole-line tiles (measured slower on 64-byte tiles)
                return with_nt(g.nt && xg <= 1, [&](auto ntc) -> hipError_t {
                    constexpr bool NT = decltype(ntc)::value;
                    const AxisMap am = y_map(g);
                    if (dir < 0)
                        hipLaunchKernelGGL((axis_c2c_kernel<T, PL, WM, -1, 1, NT, TL::G>), grid, block, 0, s, data,
                                           data, W, g.M, am, tiles, tw + g.tw_y, g.lt_shift, xg);
                    else
                        hipLaunchKernelGGL((axis_c2c_kernel<T, PL, WM, +1, 1, NT, TL::G>), grid, block, 0, s, data,
                                           data, W, g.M, am, tiles, tw + g.tw_y, g.lt_shift, xg);
                    return hipGetLastError();
                });
            });
        }
    });
}

template <typename T>
hipError_t launch_last_fwd(const Geom &g, const cx<T> *src, cx<T> *dst, const cx<T> *tw, hipStream_t s)
{
    return launch_last_c2c<T>(g, src, dst, -1, tw, s);
}

template <typename T>
hipError_t launch_last_c2c(const Geom &g, const cx<T> *src, cx<T> *dst, int dir, const cx<T> *tw, hipStream_t s)
{
    if (!layout_ok(g)) return hipErrorInvalidValue;
    return by_length(g.n0, [&](auto Lc) -> hipError_t {
        constexpr int L = decltype(Lc)::value;
        if constexpr (L < 4) {
            return hipErrorInvalidValue;
        } else {
            using PL = typename AxisPlan<L>::type;
            if (!z_steps_ok<PL>(g.zs)) return hipErrorInvalidValue;
            constexpr int WM = WMax<T, L>::value;
            const int64_t ncols = g.nrows * g.M;
            const int W = (int)(ncols < WM ? ncols : WM);
            const int64_t tiles = cdiv(ncols, W);
            const dim3 grid((unsigned)tiles), block(WM * PL::Tp);
            const AxisMap am = last_map(g);
            if (dir < 0)
                hipLaunchKernelGGL((axis_c2c_kernel<T, PL, WM, -1>), grid, block, 0, s, src, dst, W, ncols, am, tiles,
                                   tw + g.tw_last, g.lt_shift, 1);
            else
                hipLaunchKernelGGL((axis_c2c_kernel<T, PL, WM, +1>), grid, block, 0, s, src, dst, W, ncols, am, tiles,
                                   tw + g.tw_last, g.lt_shift, 1);
            return hipGetLastError();
        }
    });
}

template <typename T>
hipError_t launch_last_c2c_deriv(const Geom &g, const cx<T> *src, cx<T> *dst, int role, double fk, const cx<T> *tw,
                                 hipStream_t s)
{
    if (!layout_ok(g)) return hipErrorInvalidValue;
    return by_length(g.n0, [&](auto Lc) -> hipError_t {
        constexpr int L = decltype(Lc)::value;
        if constexpr (L < 4) {
            return hipErrorInvalidValue;
        } else {
            using PL = typename AxisPlan<L>::type;
            if (!z_steps_ok<PL>(g.zs)) return hipErrorInvalidValue;
            constexpr int WM = WMax<T, L>::value;
            const int64_t ncols = g.nrows * g.M;
            const int W = (int)(ncols < WM ? ncols : WM);
            const int64_t tiles = cdiv(ncols, W);
            const DerivArgs da{role, fk, g.nrows, g.M};
            hipLaunchKernelGGL((axis_c2c_deriv_kernel<T, PL, WM>), dim3((unsigned)tiles), dim3(WM * PL::Tp), 0, s, src,
                               dst, W, ncols, last_map(g), tw + g.tw_last, g.lt_shift, da);
            return hipGetLastError();
        }
    });
}

template <typename T>
hipError_t launch_last(const Geom &g, int mode, const cx<T> *src, cx<T> *dst, cx<T> *dst2, cx<T> *state,
                       const ModelParams<T> &mp, const cx<T> *tw, hipStream_t s, int variant)
{
    if (!layout_ok(g)) return hipErrorInvalidValue;
    return by_length(g.n0, [&](auto Lc) -> hipError_t {
        constexpr int L = decltype(Lc)::value;
        if constexpr (L < 4) {
            return hipErrorInvalidValue;
        } else {
            constexpr int WM = WMax<T, L>::value;
            LastAxisArgs<T> a{};
            a.src = src;
            a.dst = dst;
            a.dst2 = dst2;
            a.state = state;
            a.nrows = g.nrows;
            a.M = (int)g.M;
            // even tile width: the pair tiles split it between the rows k_y and -k_y
            a.W = even_width(g.M < WM ? (int)g.M : WM);
            a.tiles_per_row = (int)cdiv(g.M, a.W);
            a.tw = tw + g.tw_last;
            a.lt_shift = g.lt_shift;
            a.mp = mp;
            a.pk = pack_of(g);
            a.pk2 = Pack{g.nrows, g.M, 0, 0};  // ADJOINT's nu: plain rows of M
            const int64_t nblocks = (g.nrows == 1) ? a.tiles_per_row : g.nrows * a.tiles_per_row;
            const dim3 grid((unsigned)nblocks);
            using P0 = typename LastPlan<L>::type;
            if (mode != LAST_STEP && !z_steps_ok<P0>(g.zs)) return hipErrorInvalidValue;
            switch (mode) {
            case LAST_STEP: {
                auto run = [&](auto plc) -> hipError_t {
                    using TO = TileOf<T, decltype(plc)>;
                    using TL = typename TO::tile;
                    using PL = SpreadIf<typename TO::plan, TL::E>;
                    if (!z_steps_ok<PL>(g.zs)) return hipErrorInvalidValue;
                    LastAxisArgs<T> b = a;
                    b.W = even_width(g.M < TL::W ? (int)g.M : TL::W);
                    b.tiles_per_row = (int)cdiv(g.M, b.W);
                    const int64_t nb = (g.nrows == 1) ? b.tiles_per_row : g.nrows * b.tiles_per_row;
                    return with_nt(g.nt && line_group<T>(b.W) == 1, [&](auto ntc) -> hipError_t {
                        hipLaunchKernelGGL((last_axis_kernel<T, PL, TL::W, LA_STEP, 1, TL::PF, ORD_XCD_ROW,
                                                             decltype(ntc)::value, TL::G>),
                                           dim3((unsigned)nb), dim3(TL::W * PL::Tp), 0, s, b);
                        return hipGetLastError();
                    });
                };
                // 3D: the z candidates (wider tiles at some lengths); 2D: the list the batched
                // kernel shares, so that its instances stay bitwise equal to single plans
                if (g.ndim == 3) return with_plan<typename ZCandsOf<T, L>::type>(variant, run);
                return with_plan<typename LastCands<L>::type>(variant, run);
            }
            // natural layout (rows of M + 1, not line-aligned): whole rows per XCD, so the lines two
            // tiles share meet in one L2 (measured at 512^3: r2c 403 -> 348 us, c2r 274 -> 262 us)
            case LAST_R2C_NATURAL: {
                // line-aligned output chunks where the geometry allows (3D r2c at 512^3 FP32: 0.734 ->
                // 0.660 ms against the tiles below), else column tiles in whole rows per XCD
                using TL = PencilTile<T, L>;
                constexpr int C = 128 / (int)sizeof(cx<T>);
                if constexpr (TL::W == C && L <= 1024) {  // at 2048 the two rounds' registers would spill
                    if (g.nrows > 1 && (g.nrows * (g.M + 1)) % C == 0 && g.M >= C) {
                        using PL = SpreadIf<P0, TL::E>;
                        if (!z_steps_ok<PL>(g.zs)) return hipErrorInvalidValue;
                        const int64_t nchunks = g.nrows * (g.M + 1) / C;
                        return with_nt(g.nt, [&](auto ntc) -> hipError_t {
                            hipLaunchKernelGGL((r2c_natural_chunk_kernel<T, PL, C, TL::G, decltype(ntc)::value>),
                                               dim3((unsigned)nchunks), dim3(C * PL::Tp), 0, s, src, dst, g.nrows,
                                               (int)g.M, tw + g.tw_last, g.lt_shift, pack_of(g));
                            return hipGetLastError();
                        });
                    }
                }
                hipLaunchKernelGGL((last_axis_kernel<T, P0, WM, LA_R2C_NATURAL, 1, true, ORD_XCD_ROW>), grid,
                                   dim3(WM * P0::Tp), 0, s, a);
                break;
            }
            case LAST_C2R_NATURAL:
                return with_nt(g.nt && line_group<T>(a.W) == 1, [&](auto ntc) -> hipError_t {
                    hipLaunchKernelGGL(
                        (last_axis_kernel<T, P0, WM, LA_C2R_NATURAL, 1, true, ORD_XCD_ROW, decltype(ntc)::value>), grid,
                        dim3(WM * P0::Tp), 0, s, a);
                    return hipGetLastError();
                });
            case LAST_ADJOINT:
                hipLaunchKernelGGL((last_axis_kernel<T, P0, WM, LA_ADJOINT>), grid, dim3(WM * P0::Tp), 0, s, a);
                break;
            default: return hipErrorInvalidValue;
            }
            return hipGetLastError();
        }
    });
}

template <typename T>
hipError_t launch_set_mass(const T *psi, int64_t n, double *partial, cx<T> *state, hipStream_t s)
{
    hipLaunchKernelGGL((sum_kernel<T>), dim3(kReduceBlocks), dim3(256), 0, s, psi, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((set_mass_kernel<T>), dim3(1), dim3(64), 0, s, partial, kReduceBlocks, state);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_energy(const Geom &g, const T *psi, const cx<T> *state, const double fk[3], double r, double q1sq,
                         double R1, int model, double dV, double *partial, double *out, hipStream_t s)
{
    if (!layout_ok(g)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((energy_spec_kernel<T>), dim3(kReduceBlocks), dim3(256), 0, s, state, g.n0, g.nrows, g.M,
                       fk[0], fk[1], fk[2], r, q1sq, R1, model, partial, pack_of(g));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t ntot = g.n0 * g.nrows * g.nx;
    hipLaunchKernelGGL((quartic_kernel<T>), dim3(kReduceBlocks), dim3(256), 0, s, psi, ntot, partial + kReduceBlocks);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((energy_final_kernel<T>), dim3(1), dim3(64), 0, s, partial, partial + kReduceBlocks,
                       kReduceBlocks, dV, (double)ntot, state, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_export(const Geom &g, const cx<T> *state, cx<T> *out, hipStream_t s)
{
    if (!layout_ok(g)) return hipErrorInvalidValue;
    const int64_t n = g.n0 * g.nrows * (g.M + 1);
    const int64_t blocks = cdiv(n, 256) < 65536 ? cdiv(n, 256) : 65536;
    hipLaunchKernelGGL((export_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, s, state, out, g.n0, g.nrows, g.M,
                       pack_of(g));
    return hipGetLastError();
}

#define PFC_INSTANTIATE(T)                                                                                            \
    template hipError_t launch_x_r2c<T>(const Geom &, const T *, cx<T> *, bool, const cx<T> *, hipStream_t, int);     \
    template hipError_t launch_x_c2r<T>(const Geom &, const cx<T> *, T *, const cx<T> *, hipStream_t, int);           \
    template hipError_t launch_x_c2r_r2c<T>(const Geom &, cx<T> *, const cx<T> *, hipStream_t);                        \
    template bool x_fused_ok<T>(const Geom &);                                                                        \
    template bool z_blocks_ok<T>(const Geom &, int);                                                                  \
    template hipError_t launch_x_c2r_adjoint<T>(const Geom &, const cx<T> *, const cx<T> *, const T *, const T *, T *, \
                                                T, double *, int64_t *, const cx<T> *, hipStream_t);                  \
    template hipError_t launch_y_c2c<T>(const Geom &, cx<T> *, int, const cx<T> *, hipStream_t, int);                 \
    template hipError_t launch_last_fwd<T>(const Geom &, const cx<T> *, cx<T> *, const cx<T> *, hipStream_t);         \
    template hipError_t launch_last_c2c<T>(const Geom &, const cx<T> *, cx<T> *, int, const cx<T> *, hipStream_t);    \
    template hipError_t launch_last_c2c_deriv<T>(const Geom &, const cx<T> *, cx<T> *, int, double, const cx<T> *,    \
                                                 hipStream_t);                                                        \
    template hipError_t launch_x_c2r_mac<T>(const Geom &, const cx<T> *, T *, const T *, bool, const cx<T> *,         \
                                            hipStream_t);                                                             \
    template hipError_t launch_spec_update<T>(const Geom &, int, cx<T> *, const cx<T> *, const cx<T> *,               \
                                              const HydroArgs &, hipStream_t);                                        \
    template hipError_t launch_last<T>(const Geom &, int, const cx<T> *, cx<T> *, cx<T> *, cx<T> *,                   \
                                       const ModelParams<T> &, const cx<T> *, hipStream_t, int);                      \
    template hipError_t launch_set_mass<T>(const T *, int64_t, double *, cx<T> *, hipStream_t);                       \
    template hipError_t launch_energy<T>(const Geom &, const T *, const cx<T> *, const double *, double, double,      \
                                         double, int, double, double *, double *, hipStream_t);                       \
    template hipError_t launch_export<T>(const Geom &, const cx<T> *, cx<T> *, hipStream_t);

}  // namespace pfc
