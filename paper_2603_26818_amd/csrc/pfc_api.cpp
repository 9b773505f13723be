// pfc_api.cpp -- C ABI of the PFC library: plan validation, workspace, and the pass sequences of
// each entry point (see include/pfc.h for the contract of every call).
#include "../../include/pfc.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "api_internal.hpp"
#include "fft_core.hpp"
#include "apfc_launch.hpp"
#include "launch.hpp"
#include "types.hpp"

using pfc::cx;
using pfc::Geom;

struct pfc_plan {
    pfc_plan_desc d;
    Geom g;
    double fk[3];  // 2 pi / (n dx) for axes (last-axis, rows, x)
    double dV;
    size_t tw_off, partial_off, watch_off, scratch_off, ws_need;
    size_t tw_entries;  // power-of-two tables plus the own tables of non-power-of-two lengths
    size_t n_partials;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    int var[5] = {0, 0, 0, 0, 0};  // candidate schedule of each step pass (autotuner)
    bool x_fused = false;          // the geometry has the fused x pass between steps
    std::vector<char> tw_host;     // the twiddle tables as uploaded (built on first use)
    uint64_t id = 0;               // unique per plan in this process
};

struct pfc_batch {
    int count = 0;
    pfc_dtype dtype = PFC_F32;
    int device = 0;
    std::vector<pfc_plan_desc> descs;  // caller's order
    std::vector<int> order;            // device table order (largest first) -> caller's index
    struct Inst {
        int n0, nx, M, x_rows, c_rows, W, tiles, x_items, c_items, f_rows, f_items;
        int vx = 0, vy = 0, vc = 0;  // candidate schedules (autotuner)
    };
    std::vector<Inst> inst;  // caller's order
    int lt_shift = 0;
    int x_total = 0, y_total = 0, c_total = 0, f_total = 0;
    size_t ctl_off = 0, inst_off = 0, tw_off = 0, partial_off = 0, ws_need = 0;
    std::vector<size_t> scratch_off;  // caller's order
    char *ws = nullptr;
    size_t ws_bytes = 0;
    std::vector<void *> psi, state;
    int grid = 0;
    hipStream_t cap = nullptr;
    std::map<int64_t, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
};

namespace {

thread_local std::string g_last_error;

pfc_status fail(pfc_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

pfc_status hip_fail(hipError_t e, const char *what)
{
    return fail(PFC_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

size_t cx_size(const pfc_plan *p) { return p->d.dtype == PFC_F64 ? 16 : 8; }

double corr_op(const pfc_plan_desc &d, double q)
{
    double a = (1.0 - q) * (1.0 - q);
    if (d.model == PFC_ONE_MODE) return a;
    double b = d.q1sq - q;
    return a * (b * b + d.R1);
}

// The implicit denominator 1 + dt q (r + L(q)) must stay positive for every q in [0, qmax]
// (qmax = |k|^2 at the corner of the grid).  Checked on a dense sampling of the interval.
pfc_status check_denominator(const pfc_plan_desc &d)
{
    double qmax = 0.0;
    for (int a = 0; a < d.ndim; ++a) {
        double k = M_PI / d.dx[a];
        qmax += k * k;
    }
    const int ns = 1 << 18;
    double worst = INFINITY, worst_q = 0.0;
    for (int i = 0; i <= ns; ++i) {
        double q = qmax * (double)i / ns;
        double den = 1.0 + d.dt * q * (d.r + corr_op(d, q));
        if (!(den > worst)) {
            worst = den;
            worst_q = q;
        }
    }
    if (!(worst > 0.0))
        return fail(PFC_ERR_INVALID_ARG, "1 + dt q (r + L(q)) = %g <= 0 at q = %g: dt too large for this r", worst,
                    worst_q);
    return PFC_OK;
}

pfc_status validate_desc(const pfc_plan_desc *d)
{
    if (!d) return fail(PFC_ERR_INVALID_ARG, "desc is NULL");
    if (d->ndim != 2 && d->ndim != 3) return fail(PFC_ERR_UNSUPPORTED, "ndim must be 2 or 3 (got %d)", d->ndim);
    for (int a = 0; a < d->ndim; ++a) {
        // axis lengths: powers of two in [4, 2048], or even lengths whose own (y, last axis) or half
        // (x) length has a compiled mixed-radix schedule
        const int64_t n = d->n[a], L = (a == d->ndim - 1) ? n / 2 : n;
        const bool ok = (is_pow2(n) && n >= 4 && n <= 2048) || (n % 2 == 0 && n <= 2048 && pfc::mixed_length(L));
        if (!ok)
            return fail(PFC_ERR_UNSUPPORTED,
                        "n[%d] = %lld: sizes must be powers of two in [4, 2048] or even lengths with a mixed-radix "
                        "schedule",
                        a, (long long)n);
        if (!(d->dx[a] > 0.0) || !std::isfinite(d->dx[a])) return fail(PFC_ERR_INVALID_ARG, "dx[%d] must be > 0", a);
    }
    if (d->dtype != PFC_F32 && d->dtype != PFC_F64) return fail(PFC_ERR_INVALID_ARG, "unknown dtype %d", (int)d->dtype);
    if (d->model != PFC_ONE_MODE && d->model != PFC_TWO_MODE)
        return fail(PFC_ERR_INVALID_ARG, "unknown model %d", (int)d->model);
    if (!std::isfinite(d->r) || !std::isfinite(d->q1sq) || !std::isfinite(d->R1))
        return fail(PFC_ERR_INVALID_ARG, "non-finite model parameter");
    if (!(d->dt > 0.0) || !std::isfinite(d->dt)) return fail(PFC_ERR_INVALID_ARG, "dt must be > 0 and finite");
    const uint32_t known = PFC_FLAG_LINEAR_ONLY | PFC_FLAG_ZBLOCK(3) | PFC_FLAG_XROWS_BLOCK;
    if (d->flags & ~known) return fail(PFC_ERR_INVALID_ARG, "unknown flag bits 0x%x", d->flags);
    if (d->device < 0) return fail(PFC_ERR_INVALID_ARG, "device must be >= 0");
    return check_denominator(*d);
}

// exp(-2 pi i e / Lt) in extended precision, by octant symmetry so that the table is exactly
// symmetric, then rounded once to the dtype.
void twiddle_value(int64_t e, int64_t Lt, long double *c, long double *s)
{
    const long double two_pi = 6.283185307179586476925286766559005768L;
    const int64_t q4 = Lt / 4;
    e %= Lt;
    int64_t quad = e / q4, rem = e % q4;
    long double cc, ss;
    if (2 * rem <= q4) {
        long double a = two_pi * (long double)rem / (long double)Lt;
        cc = cosl(a);
        ss = sinl(a);
    } else {
        long double b = two_pi * (long double)(q4 - rem) / (long double)Lt;
        cc = sinl(b);
        ss = cosl(b);
    }
    // rotate by quad quarter turns: angle + quad * pi/2
    for (int64_t k = 0; k < quad; ++k) {
        long double t = cc;
        cc = -ss;
        ss = t;
    }
    *c = cc;
    *s = -ss;  // forward sign
}

// The twiddle buffer (layout in types.hpp): Lt entries of W_Lt^e, then the per-stage tables,
// every value rounded once from twiddle_value.
size_t twiddle_count(int64_t Lt) { return (size_t)(Lt + pfc::stage_tw_entries(Lt)); }

template <typename T>
std::vector<cx<T>> twiddle_table(int64_t Lt)
{
    std::vector<cx<T>> tw(twiddle_count(Lt));
    for (int64_t e = 0; e < Lt; ++e) {
        long double c, sn;
        twiddle_value(e, Lt, &c, &sn);
        tw[e].x = (T)c;
        tw[e].y = (T)sn;
    }
    for (int64_t Np = 2; Np <= Lt; Np *= 2)
        for (int R = 2; R <= 16 && R <= Np; R *= 2) {
            cx<T> *blk = tw.data() + Lt + pfc::stage_tw_offset(Np, R);
            for (int64_t jj = 0; jj < Np / R; ++jj)
                for (int r = 0; r < R; ++r) blk[jj * R + r] = tw[(jj * r * (Lt / Np)) % Lt];
        }
    return tw;
}

// Own twiddle table of a length L that is not a power of two (layout: MixTable in fft_core.hpp).
template <typename T>
cx<T> unit_root(int64_t m, int64_t N)  // exp(-2 pi i m / N)
{
    return {(T)pfc::cs2pi(m, N, 0), (T)(-pfc::cs2pi(m, N, 1))};
}
template <typename T, int L>
void fill_mix_table(cx<T> *out)
{
    using MT = pfc::MixTable<L>;
    auto blocks = [&](auto pc, int base) {
        using P = decltype(pc);
        for (int st = 0; st < P::nst; ++st) {
            const int Ns = P::prefix(st), R = P::radix(st);
            cx<T> *blk = out + base + pfc::stage_blocks_off<P>(st);
            for (int jj = 0; jj < Ns; ++jj)
                for (int r = 0; r < R; ++r) blk[jj * R + r] = unit_root<T>((int64_t)jj * r, (int64_t)Ns * R);
        }
    };
    blocks(typename MT::F{}, 0);
    blocks(typename MT::Rv{}, pfc::stage_blocks_off<typename MT::F>(MT::F::nst));
    for (int k = 0; k < L; ++k) out[MT::split + k] = unit_root<T>(k, 2 * (int64_t)L);
}
// calls f(std::integral_constant<int, L>) for a supported non-power-of-two length
template <class F>
bool with_mixed_length(int64_t L, F &&f)
{
    switch (L) {
#define PFC_MIXCASE(LL)                                                                                    \
    case LL: f(std::integral_constant<int, LL>{}); return true;
        PFC_MIXCASE(6) PFC_MIXCASE(10) PFC_MIXCASE(12) PFC_MIXCASE(14) PFC_MIXCASE(15) PFC_MIXCASE(20)
        PFC_MIXCASE(30) PFC_MIXCASE(60) PFC_MIXCASE(150) PFC_MIXCASE(375) PFC_MIXCASE(700) PFC_MIXCASE(750)
        PFC_MIXCASE(1400)
#undef PFC_MIXCASE
    default: return false;
    }
}
size_t mix_table_entries(int64_t L)
{
    size_t n = 0;
    with_mixed_length(L, [&](auto lc) { n = (size_t)pfc::MixTable<decltype(lc)::value>::size; });
    return (n + 1) & ~size_t(1);  // keep the next table 16-byte aligned
}

// The plan's twiddle tables as the device holds them (power-of-two tables, then the own table of
// each non-power-of-two pass length), built once per plan.
const std::vector<char> &host_tables(pfc_plan *p)
{
    if (!p->tw_host.empty()) return p->tw_host;
    const int64_t Lt = int64_t(1) << p->g.lt_shift;
    auto build = [&](auto tc) {
        using T = decltype(tc);
        std::vector<cx<T>> tw = twiddle_table<T>(Lt);
        tw.resize(p->tw_entries);
        const int64_t lens[3] = {p->g.M, p->d.ndim == 3 ? p->g.n1 : 0, p->g.n0};
        const int64_t offs[3] = {p->g.tw_x, p->g.tw_y, p->g.tw_last};
        for (int i = 0; i < 3; ++i)
            if (offs[i] > 0)
                with_mixed_length(lens[i], [&](auto lc) { fill_mix_table<T, decltype(lc)::value>(tw.data() + offs[i]); });
        p->tw_host.assign((const char *)tw.data(), (const char *)(tw.data() + tw.size()));
    };
    if (p->d.dtype == PFC_F64)
        build(double{});
    else
        build(float{});
    return p->tw_host;
}

// Grids whose state exceeds this use non-temporal loads and stores in the step and FFT passes:
// a pass's three grids then no longer fit in the 256 MB memory-side cache, and the hint keeps the
// caches from holding lines that are not read again.
constexpr size_t kNonTemporalBytes = size_t(128) << 20;

struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev)
    {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

pfc_status check_ready(const pfc_plan *p)
{
    if (!p) return fail(PFC_ERR_INVALID_ARG, "plan is NULL");
    if (!p->ws) return fail(PFC_ERR_WORKSPACE, "no workspace attached (pfc_plan_set_workspace)");
    return PFC_OK;
}

pfc_status check_ptr(const void *ptr, const char *name)
{
    if (!ptr) return fail(PFC_ERR_INVALID_ARG, "%s is NULL", name);
    if (!aligned16(ptr)) return fail(PFC_ERR_ALIGNMENT, "%s is not 16-byte aligned", name);
    return PFC_OK;
}

bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

template <typename T>
pfc::ModelParams<T> model_params(const pfc_plan *p)
{
    pfc::ModelParams<T> m;
    m.r = (T)p->d.r;
    m.dt = (T)p->d.dt;
    m.q1sq = (T)p->d.q1sq;
    m.R1 = (T)p->d.R1;
    for (int a = 0; a < 3; ++a) m.fk[a] = (T)p->fk[a];
    m.nl = (p->d.flags & PFC_FLAG_LINEAR_ONLY) ? T(0) : T(1);
    m.model = (int)p->d.model;
    return m;
}

template <typename T>
struct Bufs {
    const cx<T> *tw;
    double *partial;
    cx<T> *scratch;
};

template <typename T>
Bufs<T> bufs(const pfc_plan *p)
{
    return {reinterpret_cast<const cx<T> *>(p->ws + p->tw_off), reinterpret_cast<double *>(p->ws + p->partial_off),
            reinterpret_cast<cx<T> *>(p->ws + p->scratch_off)};
}

#define PFC_TRY(call, what)                           \
    do {                                              \
        hipError_t e_ = (call);                       \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// forward transform of a real field into the packed spectrum `out` (x, then y in 3D; the last
// axis is left to the caller)
template <typename T>
pfc_status fwd_xy(const pfc_plan *p, const T *real, bool cube, cx<T> *out, hipStream_t s)
{
    const Geom &g = p->g;
    const Bufs<T> b = bufs<T>(p);
    PFC_TRY(pfc::launch_x_r2c<T>(g, real, out, cube, b.tw, s), "x_r2c launch");
    if (g.ndim == 3) PFC_TRY(pfc::launch_y_c2c<T>(g, out, -1, b.tw, s), "y forward launch");
    return PFC_OK;
}

template <typename T>
pfc_status inv_yx(const pfc_plan *p, cx<T> *spec, T *real, hipStream_t s)
{
    const Geom &g = p->g;
    const Bufs<T> b = bufs<T>(p);
    if (g.ndim == 3) PFC_TRY(pfc::launch_y_c2c<T>(g, spec, +1, b.tw, s), "y inverse launch");
    PFC_TRY(pfc::launch_x_c2r<T>(g, spec, real, b.tw, s), "x_c2r launch");
    return PFC_OK;
}

template <typename T>
pfc_status do_r2c(pfc_plan *p, const void *in, void *out, hipStream_t s)
{
    const Bufs<T> b = bufs<T>(p);
    pfc_status st = fwd_xy<T>(p, (const T *)in, false, b.scratch, s);
    if (st) return st;
    pfc::ModelParams<T> mp = model_params<T>(p);
    PFC_TRY(pfc::launch_last<T>(p->g, pfc::LAST_R2C_NATURAL, b.scratch, (cx<T> *)out, nullptr, nullptr, mp, b.tw, s),
            "last-axis launch");
    return PFC_OK;
}

template <typename T>
pfc_status do_c2r(pfc_plan *p, const void *in, void *out, hipStream_t s)
{
    const Bufs<T> b = bufs<T>(p);
    pfc::ModelParams<T> mp = model_params<T>(p);
    PFC_TRY(pfc::launch_last<T>(p->g, pfc::LAST_C2R_NATURAL, (const cx<T> *)in, b.scratch, nullptr, nullptr, mp, b.tw,
                                s),
            "last-axis launch");
    return inv_yx<T>(p, b.scratch, (T *)out, s);
}

template <typename T>
pfc_status do_state_init(pfc_plan *p, const void *psi0, void *state, hipStream_t s)
{
    const Bufs<T> b = bufs<T>(p);
    pfc_status st = fwd_xy<T>(p, (const T *)psi0, false, b.scratch, s);
    if (st) return st;
    PFC_TRY(pfc::launch_last_fwd<T>(p->g, b.scratch, (cx<T> *)state, b.tw, s), "last-axis launch");
    const int64_t ntot = p->g.n0 * p->g.nrows * p->g.nx;
    PFC_TRY(pfc::launch_set_mass<T>((const T *)psi0, ntot, b.partial, (cx<T> *)state, s), "mass launch");
    return PFC_OK;
}

// One pass of a step.  3D: 0 x r2c + cube, 1 y forward, 2 z fused update, 3 y inverse, 4 x c2r.
// 2D: 0 x r2c + cube, 1 y fused update, 2 x c2r.
int step_passes(const pfc_plan *p) { return p->g.ndim == 3 ? 5 : 3; }

template <typename T>
pfc_status step_pass(const pfc_plan *p, const Bufs<T> &b, int pass, void *psi, void *state, hipStream_t s)
{
    const Geom &g = p->g;
    const int id = (g.ndim == 3) ? pass : (pass == 0 ? 0 : pass == 1 ? 2 : 4);
    const int v = p->var[pass];
    switch (id) {
    case 0: PFC_TRY(pfc::launch_x_r2c<T>(g, (const T *)psi, b.scratch, true, b.tw, s, v), "x_r2c launch"); break;
    case 1: PFC_TRY(pfc::launch_y_c2c<T>(g, b.scratch, -1, b.tw, s, v), "y forward launch"); break;
    case 2: {
        const pfc::ModelParams<T> mp = model_params<T>(p);
        PFC_TRY(pfc::launch_last<T>(g, pfc::LAST_STEP, b.scratch, b.scratch, nullptr, (cx<T> *)state, mp, b.tw, s, v),
                "last-axis step launch");
        break;
    }
    case 3: PFC_TRY(pfc::launch_y_c2c<T>(g, b.scratch, +1, b.tw, s, v), "y inverse launch"); break;
    case 4: PFC_TRY(pfc::launch_x_c2r<T>(g, b.scratch, (T *)psi, b.tw, s, v), "x_c2r launch"); break;
    default: return fail(PFC_ERR_INTERNAL, "bad pass %d", pass);
    }
    return PFC_OK;
}

// Steps in sequence.  Between two steps the x c2r of the first and the x r2c (with the cube) of the
// second run as one fused pass on the spectrum (launch_x_c2r_r2c: the real field in between stays in
// LDS and is never stored), where the geometry has it and both x passes take their default schedules;
// the first step's x r2c reads psi and the last step's x c2r writes it.  The results are those of
// the separate passes, bit for bit.
template <typename T>
pfc_status step_with(const pfc_plan *p, const Bufs<T> &b, void *psi, void *state, int64_t nsteps, hipStream_t s)
{
    const int np = step_passes(p);
    const bool fuse = p->x_fused && p->var[0] == 0 && p->var[np - 1] == 0;
    for (int64_t n = 0; n < nsteps; ++n)
        for (int k = 0; k < np; ++k) {
            if (fuse && k == 0 && n > 0) continue;  // done by the fused pass that ended the step before
            if (fuse && k == np - 1 && n + 1 < nsteps) {
                PFC_TRY(pfc::launch_x_c2r_r2c<T>(p->g, b.scratch, b.tw, s), "fused x pass launch");
                continue;
            }
            pfc_status st = step_pass<T>(p, b, k, psi, state, s);
            if (st) return st;
        }
    return PFC_OK;
}

template <typename T>
pfc_status do_step(pfc_plan *p, void *psi, void *state, int64_t nsteps, hipStream_t s)
{
    return step_with<T>(p, bufs<T>(p), psi, state, nsteps, s);
}

template <typename T>
pfc_status do_step_timed(pfc_plan *p, void *psi, void *state, int64_t nsteps, hipStream_t s, double *pass_ms)
{
    const int np = step_passes(p);
    hipEvent_t ev[6];
    int made = 0;
    pfc_status st = PFC_OK;
    for (; made < np + 1; ++made) {
        hipError_t e = hipEventCreate(&ev[made]);
        if (e != hipSuccess) {
            st = hip_fail(e, "hipEventCreate");
            break;
        }
    }
    for (int k = 0; k < np; ++k) pass_ms[k] = 0.0;
    for (int64_t n = 0; n < nsteps && st == PFC_OK; ++n) {
        hipError_t e = hipEventRecord(ev[0], s);
        for (int k = 0; k < np && e == hipSuccess && st == PFC_OK; ++k) {
            st = step_pass<T>(p, bufs<T>(p), k, psi, state, s);
            if (st == PFC_OK) e = hipEventRecord(ev[k + 1], s);
        }
        if (st == PFC_OK && e == hipSuccess) e = hipEventSynchronize(ev[np]);
        for (int k = 0; k < np && st == PFC_OK && e == hipSuccess; ++k) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
            pass_ms[k] += ms;
        }
        if (st == PFC_OK && e != hipSuccess) st = hip_fail(e, "timing events");
    }
    for (int k = 0; k < made; ++k) (void)hipEventDestroy(ev[k]);
    return st;
}

// Times every candidate schedule of every step pass (`reps` launches each after one warm-up,
// events on the stream) and keeps the fastest.  psi/state are scratch: their contents change.
template <typename T>
pfc_status do_autotune(pfc_plan *p, void *psi, void *state, hipStream_t s, int reps, double *best_ms)
{
    hipEvent_t e0, e1;
    PFC_TRY(hipEventCreate(&e0), "hipEventCreate");
    hipError_t ce = hipEventCreate(&e1);
    if (ce != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(ce, "hipEventCreate");
    }
    pfc_status st = PFC_OK;
    const int np = step_passes(p);
    // elapsed ms of `fn` run `n` times on the stream, after one untimed run
    auto timed = [&](int n, auto &&fn, float *ms) -> pfc_status {
        pfc_status r = fn();
        hipError_t e = hipEventRecord(e0, s);
        for (int i = 0; i < n && r == PFC_OK && e == hipSuccess; ++i) r = fn();
        if (r == PFC_OK && e == hipSuccess) e = hipEventRecord(e1, s);
        if (r == PFC_OK && e == hipSuccess) e = hipEventSynchronize(e1);
        if (r == PFC_OK && e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
        if (r == PFC_OK && e != hipSuccess) r = hip_fail(e, "autotune timing");
        return r;
    };
    // Coordinate descent over whole steps: from the default schedules, each candidate of each pass in
    // turn is kept when a run of steps with it is faster.  Timing a pass alone, repeated on the same
    // data, misjudges it (at 512^3 FP32 such per-pass choices made the step 1.6 % slower), and whole
    // steps include the fused x pass between steps, which runs on the default x schedules only.
    const int64_t k_steps = 4;
    auto run = [&] { return step_with<T>(p, bufs<T>(p), psi, state, k_steps, s); };
    for (int k = 0; k < np; ++k) p->var[k] = 0;
    float t_best = 0.f;
    st = timed(reps, run, &t_best);
    for (int k = 0; k < np && st == PFC_OK; ++k) {
        const int nc = pfc::step_candidates(p->g, k);
        int best = 0;
        for (int c = 1; c < nc && st == PFC_OK; ++c) {
            p->var[k] = c;
            float ms = 0.f;
            st = timed(reps, run, &ms);
            if (st == PFC_OK && ms < t_best) {
                t_best = ms;
                best = c;
            }
        }
        p->var[k] = best;
    }
    // per-pass times of the choice (the passes apart, as pfc_step_timed runs them)
    if (st == PFC_OK && best_ms) {
        double pm[5] = {};
        st = do_step_timed<T>(p, psi, state, reps, s, pm);
        for (int k = 0; k < np && st == PFC_OK; ++k) best_ms[k] = pm[k] / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

template <typename T>
pfc_status do_backward(pfc_plan *p, const void *psi_n, const void *psi_np1, const void *lam_np1, void *lam_n,
                       double *dLdr, hipStream_t s)
{
    const Geom &g = p->g;
    const Bufs<T> b = bufs<T>(p);
    const pfc::ModelParams<T> mp = model_params<T>(p);
    pfc_status st = fwd_xy<T>(p, (const T *)lam_np1, false, b.scratch, s);
    if (st) return st;
    // The output buffer holds the nu spectrum until the last pass.  nu is kept in the plain layout
    // (rows of M, no plane blocks), where its row r covers exactly the bytes of the real row r, so
    // the last pass can read each row of nu before it overwrites the same bytes with lambda_n.
    cx<T> *nu = (cx<T> *)lam_n;
    Geom gn = g;
    gn.Mp = g.M;
    gn.zs = 0;
    PFC_TRY(pfc::launch_last<T>(g, pfc::LAST_ADJOINT, b.scratch, b.scratch, nu, nullptr, mp, b.tw, s),
            "last-axis adjoint launch");
    if (g.ndim == 3) {
        PFC_TRY(pfc::launch_y_c2c<T>(g, b.scratch, +1, b.tw, s), "y inverse launch");
        PFC_TRY(pfc::launch_y_c2c<T>(gn, nu, +1, b.tw, s), "y inverse launch");
    }
    const T c3 = (p->d.flags & PFC_FLAG_LINEAR_ONLY) ? T(0) : (T)(3.0 * p->d.dt);
    int64_t nb = 0;
    PFC_TRY(pfc::launch_x_c2r_adjoint<T>(g, b.scratch, nu, (const T *)psi_n, (const T *)psi_np1, (T *)lam_n, c3,
                                          b.partial, &nb, b.tw, s),
            "x_c2r adjoint launch");
    if ((size_t)nb > p->n_partials) return fail(PFC_ERR_INTERNAL, "partials buffer too small");
    PFC_TRY(pfc::launch_accumulate(b.partial, (int)nb, -p->d.dt, dLdr, s), "accumulate launch");
    return PFC_OK;
}

template <typename T>
pfc_status do_energy(pfc_plan *p, const void *psi, const void *state, double *out, hipStream_t s)
{
    const Bufs<T> b = bufs<T>(p);
    PFC_TRY(pfc::launch_energy<T>(p->g, (const T *)psi, (const cx<T> *)state, p->fk, p->d.r, p->d.q1sq, p->d.R1,
                                  (int)p->d.model, p->dV, b.partial, out, s),
            "energy launch");
    return PFC_OK;
}

template <typename T>
pfc_status do_step_watched(pfc_plan *p, void *psi, void *state, int64_t nsteps, int64_t every, hipStream_t s,
                           int64_t *done)
{
    *done = 0;
    double *dev = reinterpret_cast<double *>(p->ws + p->watch_off);
    while (*done < nsteps) {
        const int64_t k = std::min<int64_t>(every, nsteps - *done);
        pfc_status st = do_step<T>(p, psi, state, k, s);
        if (st) return st;
        *done += k;
        st = do_energy<T>(p, psi, state, dev, s);
        if (st) return st;
        double host[2];
        PFC_TRY(hipMemcpyAsync(host, dev, sizeof host, hipMemcpyDeviceToHost, s), "energy copy");
        PFC_TRY(hipStreamSynchronize(s), "stream synchronize");
        if (!std::isfinite(host[0]) || !std::isfinite(host[1]))
            return fail(PFC_ERR_DIVERGED, "non-finite energy (%g) or mean (%g) after %lld steps", host[0], host[1],
                        (long long)*done);
    }
    return PFC_OK;
}

template <typename T>
pfc_status do_export(pfc_plan *p, const void *state, void *out, hipStream_t s)
{
    PFC_TRY(pfc::launch_export<T>(p->g, (const cx<T> *)state, (cx<T> *)out, s), "export launch");
    return PFC_OK;
}

size_t real_bytes(const pfc_plan *p) { return (size_t)(p->g.n0 * p->g.nrows * p->g.nx) * cx_size(p) / 2; }
size_t half_bytes(const pfc_plan *p) { return (size_t)(p->g.n0 * p->g.nrows * (p->g.M + 1)) * cx_size(p); }
size_t state_bytes(const pfc_plan *p) { return (size_t)(p->g.n0 * p->g.nrows * p->g.Mp) * cx_size(p); }

// ---- hydrodynamic PFC
size_t hydro_work_bytes(const pfc_plan *p) { return 2 * align256(state_bytes(p)) + 2 * align256(real_bytes(p)); }

template <typename T>
pfc_status do_hydro_state_init(pfc_plan *p, const void *psi, void *psi_state, const void *v, void *v_state,
                               hipStream_t s)
{
    pfc_status st = do_state_init<T>(p, psi, psi_state, s);
    for (int j = 0; j < p->g.ndim && !st; ++j)
        st = do_state_init<T>(p, (const char *)v + j * real_bytes(p), (char *)v_state + j * state_bytes(p), s);
    return st;
}

// One step after another as stated with pfc_hydro_step in pfc.h, composed of the transform passes
// (x r2c, y, last axis, x c2r) and the pointwise spectral kernels.  Buffers: A, B packed spectra
// and a, h real fields in `work`; the plan's own scratch is not used.
template <typename T>
pfc_status do_hydro_step(pfc_plan *p, const pfc_hydro_params *hp, void *psi_v, void *S_v, void *v_v, void *V_v,
                         void *work, int64_t nsteps, hipStream_t s)
{
    const Geom &g = p->g;
    const Bufs<T> b = bufs<T>(p);
    const int d = g.ndim;
    const size_t sb = state_bytes(p), rb = real_bytes(p);
    char *w = (char *)work;
    cx<T> *A = (cx<T> *)w, *B = (cx<T> *)(w + align256(sb));
    T *a = (T *)(w + 2 * align256(sb)), *h = (T *)(w + 2 * align256(sb) + align256(rb));
    T *psi = (T *)psi_v;
    cx<T> *S = (cx<T> *)S_v;
    auto vj = [&](int j) { return (T *)((char *)v_v + j * rb); };
    auto Vj = [&](int j) { return (cx<T> *)((char *)V_v + j * sb); };
    pfc::HydroArgs ha;
    for (int i = 0; i < 3; ++i) ha.fk[i] = p->fk[i];
    ha.r = p->d.r;
    ha.dt = p->d.dt;
    ha.q1sq = p->d.q1sq;
    ha.R1 = p->d.R1;
    ha.nl = (p->d.flags & PFC_FLAG_LINEAR_ONLY) ? 0.0 : 1.0;
    ha.model = (int)p->d.model;
    ha.c = p->d.dt / hp->rho0;
    ha.gamma = hp->gamma;
    ha.a0 = hp->a0;
    // grid axis j -> (role of the spectral index, its wavenumber step)
    auto role = [&](int j) { return d == 3 ? j : (j == 0 ? 0 : 2); };
    auto fwd = [&](const T *real, bool cube, cx<T> *out) -> pfc_status {
        pfc_status st = fwd_xy<T>(p, real, cube, out, s);
        if (st) return st;
        PFC_TRY(pfc::launch_last_c2c<T>(g, out, out, -1, b.tw, s), "last-axis forward launch");
        return PFC_OK;
    };
    // inverse of spectrum `spec` through B into the real field `out`: plain, or out = w x (+ out)
    auto inv = [&](const cx<T> *spec, T *out, const T *wf, bool add) -> pfc_status {
        PFC_TRY(pfc::launch_last_c2c<T>(g, spec, B, +1, b.tw, s), "last-axis inverse launch");
        if (d == 3) PFC_TRY(pfc::launch_y_c2c<T>(g, B, +1, b.tw, s), "y inverse launch");
        if (wf)
            PFC_TRY(pfc::launch_x_c2r_mac<T>(g, B, out, wf, add, b.tw, s), "x_c2r launch");
        else
            PFC_TRY(pfc::launch_x_c2r<T>(g, B, out, b.tw, s), "x_c2r launch");
        return PFC_OK;
    };
    // the same for the spectral derivative i k_j of `spec`, applied as the last-axis pass loads it
    auto inv_deriv = [&](const cx<T> *spec, int j, T *out, const T *wf, bool add) -> pfc_status {
        PFC_TRY(pfc::launch_last_c2c_deriv<T>(g, spec, B, role(j), p->fk[role(j)], b.tw, s),
                "last-axis derivative inverse launch");
        if (d == 3) PFC_TRY(pfc::launch_y_c2c<T>(g, B, +1, b.tw, s), "y inverse launch");
        if (wf)
            PFC_TRY(pfc::launch_x_c2r_mac<T>(g, B, out, wf, add, b.tw, s), "x_c2r launch");
        else
            PFC_TRY(pfc::launch_x_c2r<T>(g, B, out, b.tw, s), "x_c2r launch");
        return PFC_OK;
    };
    pfc_status st = PFC_OK;
#define PFC_HY(call)        \
    do {                    \
        st = (call);        \
        if (st) return st;  \
    } while (0)
    for (int64_t n = 0; n < nsteps; ++n) {
        // density: A = FFT(psi^3), a = sum_j v_j IFFT(D_j S), B = FFT(a), S update, psi = IFFT(S)
        PFC_HY(fwd(psi, true, A));
        for (int j = 0; j < d; ++j) PFC_HY(inv_deriv(S, j, a, vj(j), j > 0));
        PFC_HY(fwd(a, false, B));
        PFC_TRY(pfc::launch_spec_update<T>(g, pfc::HYDRO_PSI, S, A, B, ha, s), "density update launch");
        PFC_HY(inv(S, psi, nullptr, false));
        // velocity: A = mu = FFT(psi^3) + (r + L) S; per component h = psi IFFT(D_j mu), B = FFT(h)
        PFC_HY(fwd(psi, true, A));
        PFC_TRY(pfc::launch_spec_update<T>(g, pfc::HYDRO_MU, A, S, (const cx<T> *)nullptr, ha, s), "mu launch");
        for (int j = 0; j < d; ++j) {
            PFC_HY(inv_deriv(A, j, h, psi, false));
            PFC_HY(fwd(h, false, B));
            PFC_TRY(pfc::launch_spec_update<T>(g, pfc::HYDRO_VEL, Vj(j), B, (const cx<T> *)nullptr, ha, s),
                    "velocity update launch");
            PFC_HY(inv(Vj(j), vj(j), nullptr, false));
        }
    }
#undef PFC_HY
    return PFC_OK;
}


void drop_graphs(pfc_batch *b)
{
    for (auto &kv : b->graphs) {
        (void)hipGraphExecDestroy(kv.second.second);
        (void)hipGraphDestroy(kv.second.first);
    }
    b->graphs.clear();
}

// rows / pencils / items of every instance for its current candidate schedules
pfc_status batch_layout(pfc_batch *b)
{
    for (int i = 0; i < b->count; ++i) {
        pfc_batch::Inst &g = b->inst[i];
        int wm = 0;
        if (!pfc::batch_tiles(g.n0, g.M, g.vx, g.vy, g.vc, b->dtype == PFC_F64, &g.x_rows, &g.c_rows, &wm))
            return fail(PFC_ERR_UNSUPPORTED, "instance %d: no batched schedule for %d x %d (candidates %d %d %d)", i,
                        g.n0, g.nx, g.vx, g.vy, g.vc);
        g.W = std::min(wm, g.M);
        g.tiles = g.M / g.W;
        g.x_items = (g.n0 + g.x_rows - 1) / g.x_rows;
        g.c_items = (g.n0 + g.c_rows - 1) / g.c_rows;
        g.f_rows = std::max(g.x_rows, g.c_rows);  // both powers of two: a multiple of each
        if (g.f_rows % g.x_rows || g.f_rows % g.c_rows)
            return fail(PFC_ERR_INTERNAL, "instance %d: rows per item %d and %d do not nest", i, g.x_rows, g.c_rows);
        g.f_items = (g.n0 + g.f_rows - 1) / g.f_rows;
    }
    return PFC_OK;
}

// builds the device instance table (largest instances first) and uploads it (synchronous)
template <typename T>
pfc_status batch_upload_table(pfc_batch *b)
{
    std::vector<pfc::BatchInst<T>> table(b->count);
    int xb = 0, yb = 0, cb = 0, fb = 0;
    for (int j = 0; j < b->count; ++j) {
        const int i = b->order[j];
        const pfc_batch::Inst &g = b->inst[i];
        const pfc_plan_desc &d = b->descs[i];
        pfc::BatchInst<T> &t = table[j];
        t.psi = (T *)b->psi[i];
        t.state = (cx<T> *)b->state[i];
        t.scratch = (cx<T> *)(b->ws + b->scratch_off[i]);
        t.n0 = g.n0;
        t.M = g.M;
        t.W = g.W;
        t.tiles = g.tiles;
        t.x_items = g.x_items;
        t.c_items = g.c_items;
        t.x_rows = g.x_rows;
        t.c_rows = g.c_rows;
        t.f_rows = g.f_rows;
        t.f_items = g.f_items;
        t.x_begin = xb;
        t.y_begin = yb;
        t.c_begin = cb;
        t.f_begin = fb;
        t.vx = g.vx;
        t.vy = g.vy;
        t.vc = g.vc;
        xb += g.x_items;
        yb += g.tiles;
        cb += g.c_items;
        fb += g.f_items;
        t.sc = (T)(1.0 / ((double)g.n0 * (double)g.M));
        t.mp.r = (T)d.r;
        t.mp.dt = (T)d.dt;
        t.mp.q1sq = (T)d.q1sq;
        t.mp.R1 = (T)d.R1;
        t.mp.fk[0] = (T)(2.0 * M_PI / ((double)d.n[0] * d.dx[0]));
        t.mp.fk[1] = (T)0;
        t.mp.fk[2] = (T)(2.0 * M_PI / ((double)d.n[1] * d.dx[1]));
        t.mp.nl = (d.flags & PFC_FLAG_LINEAR_ONLY) ? T(0) : T(1);
        t.mp.model = (int)d.model;
    }
    b->x_total = xb;
    b->y_total = yb;
    b->c_total = cb;
    b->f_total = fb;
    PFC_TRY(hipMemcpy(b->ws + b->inst_off, table.data(), table.size() * sizeof(table[0]), hipMemcpyHostToDevice),
            "instance table upload");
    drop_graphs(b);  // the captured launches hold the item totals
    return PFC_OK;
}

template <typename T>
pfc_status batch_bind_impl(pfc_batch *b)
{
    pfc_status st = batch_upload_table<T>(b);
    if (st) return st;
    const std::vector<cx<T>> tw = twiddle_table<T>(int64_t(1) << b->lt_shift);
    PFC_TRY(hipMemcpy(b->ws + b->tw_off, tw.data(), tw.size() * sizeof(tw[0]), hipMemcpyHostToDevice),
            "twiddle upload");
    PFC_TRY(hipMemset(b->ws + b->ctl_off, 0, sizeof(pfc::BatchCtl)), "barrier state reset");
    int per_cu = 0, cus = 0;
    PFC_TRY(pfc::batch_blocks_per_cu<T>(&per_cu), "occupancy query");
    PFC_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device), "CU count");
    if (per_cu < 1) return fail(PFC_ERR_INTERNAL, "batched kernel does not fit on a CU");
    b->grid = per_cu * cus;
    return PFC_OK;
}

template <typename T>
pfc::BatchArgs<T> batch_args(const pfc_batch *b, int64_t nsteps)
{
    pfc::BatchArgs<T> a;
    a.inst = (const pfc::BatchInst<T> *)(b->ws + b->inst_off);
    a.ninst = b->count;
    a.x_total = b->x_total;
    a.y_total = b->y_total;
    a.c_total = b->c_total;
    a.f_total = b->f_total;
    a.tw = (const cx<T> *)(b->ws + b->tw_off);
    a.lt_shift = b->lt_shift;
    a.ctl = (pfc::BatchCtl *)(b->ws + b->ctl_off);
    a.max_polls = 1ull << 22;  // a few seconds of polling: far beyond any pass of a resident grid
    a.nsteps = nsteps;
    return a;
}

template <typename T>
pfc_status batch_step_impl(pfc_batch *b, int64_t nsteps, hipStream_t s)
{
    auto it = b->graphs.find(nsteps);
    if (it == b->graphs.end()) {
        if (!b->cap) PFC_TRY(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking), "capture stream");
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        PFC_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal), "graph capture begin");
        hipError_t le = pfc::launch_batch<T>(batch_args<T>(b, nsteps), b->grid, b->cap);
        hipError_t ee = hipStreamEndCapture(b->cap, &graph);
        if (le != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(le, "batched kernel launch (capture)");
        }
        if (ee != hipSuccess) return hip_fail(ee, "graph capture end");
        hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return hip_fail(ie, "graph instantiate");
        }
        it = b->graphs.emplace(nsteps, std::make_pair(graph, exec)).first;
    }
    PFC_TRY(hipGraphLaunch(it->second.second, s), "graph launch");
    return PFC_OK;
}

template <typename T>
pfc_status batch_state_init_impl(pfc_batch *b, hipStream_t s)
{
    const cx<T> *tw = (const cx<T> *)(b->ws + b->tw_off);
    double *partial = (double *)(b->ws + b->partial_off);
    for (int i = 0; i < b->count; ++i) {
        const pfc_batch::Inst &in = b->inst[i];
        Geom g{};
        g.ndim = 2;
        g.n0 = in.n0;
        g.n1 = 1;
        g.nx = in.nx;
        g.M = in.M;
        g.nrows = 1;
        g.xrows = in.n0;
        g.lt_shift = b->lt_shift;
        g.nt = false;
        g.tw_x = g.tw_y = g.tw_last = 0;
        cx<T> *scratch = (cx<T> *)(b->ws + b->scratch_off[i]);
        PFC_TRY(pfc::launch_x_r2c<T>(g, (const T *)b->psi[i], scratch, false, tw, s), "x_r2c launch");
        PFC_TRY(pfc::launch_last_fwd<T>(g, scratch, (cx<T> *)b->state[i], tw, s), "last-axis launch");
        PFC_TRY(pfc::launch_set_mass<T>((const T *)b->psi[i], (int64_t)in.n0 * in.nx, partial, (cx<T> *)b->state[i], s),
                "mass launch");
    }
    return PFC_OK;
}

// Coordinate descent over the candidate schedules: for each pass kind and each distinct length,
// time every candidate by launching the persistent kernel (no graph) for `steps` steps.
template <typename T>
pfc_status batch_autotune_impl(pfc_batch *b, hipStream_t s, int steps, double *total_ms)
{
    hipEvent_t e0, e1;
    PFC_TRY(hipEventCreate(&e0), "hipEventCreate");
    hipError_t ce = hipEventCreate(&e1);
    if (ce != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(ce, "hipEventCreate");
    }
    auto trial = [&](float *ms) -> pfc_status {
        pfc_status st = batch_layout(b);
        if (!st) st = batch_upload_table<T>(b);
        if (st) return st;
        PFC_TRY(hipEventRecord(e0, s), "event record");
        PFC_TRY(pfc::launch_batch<T>(batch_args<T>(b, steps), b->grid, s), "batched kernel launch");
        PFC_TRY(hipEventRecord(e1, s), "event record");
        PFC_TRY(hipEventSynchronize(e1), "event synchronize");
        PFC_TRY(hipEventElapsedTime(ms, e0, e1), "event timing");
        pfc::BatchCtl ctl;
        PFC_TRY(hipMemcpy(&ctl, b->ws + b->ctl_off, sizeof ctl, hipMemcpyDeviceToHost), "barrier state read");
        if (ctl.err) return fail(PFC_ERR_INTERNAL, "grid barrier timed out during autotuning");
        return PFC_OK;
    };
    pfc_status st = PFC_OK;
    float ms = 0.f;
    st = trial(&ms);  // warm-up
    for (int pass = 0; pass < 3 && st == PFC_OK; ++pass) {
        std::vector<int> lens;
        for (auto &g : b->inst) lens.push_back(pass == 1 ? g.n0 : g.M);
        std::sort(lens.begin(), lens.end());
        lens.erase(std::unique(lens.begin(), lens.end()), lens.end());
        for (int len : lens) {
            const pfc_batch::Inst *any = nullptr;
            for (auto &g : b->inst)
                if ((pass == 1 ? g.n0 : g.M) == len) any = &g;
            const int nc = pfc::batch_candidates(any->n0, any->M, pass);
            int best = 0;
            float best_t = INFINITY;
            for (int c = 0; c < nc && st == PFC_OK; ++c) {
                for (auto &g : b->inst)
                    if ((pass == 1 ? g.n0 : g.M) == len) (pass == 0 ? g.vx : pass == 1 ? g.vy : g.vc) = c;
                st = trial(&ms);
                if (st == PFC_OK && ms < best_t) {
                    best_t = ms;
                    best = c;
                }
            }
            for (auto &g : b->inst)
                if ((pass == 1 ? g.n0 : g.M) == len) (pass == 0 ? g.vx : pass == 1 ? g.vy : g.vc) = best;
        }
    }
    if (st == PFC_OK) st = trial(&ms);
    if (st == PFC_OK && total_ms) *total_ms = ms / steps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

}  // namespace

extern "C" {

pfc_status pfc_plan_create(pfc_plan **out, const pfc_plan_desc *d)
{
    if (!out) return fail(PFC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    pfc_status st = validate_desc(d);
    if (st) return st;
    pfc_plan *p = new (std::nothrow) pfc_plan();
    if (!p) return fail(PFC_ERR_INTERNAL, "out of host memory");
    p->d = *d;
    static std::atomic<uint64_t> next_id{1};
    p->id = next_id.fetch_add(1);
    Geom &g = p->g;
    g.ndim = d->ndim;
    if (d->ndim == 3) {
        g.n0 = d->n[0];
        g.n1 = d->n[1];
        g.nx = d->n[2];
        g.nrows = d->n[1];
        p->fk[0] = 2.0 * M_PI / ((double)d->n[0] * d->dx[0]);
        p->fk[1] = 2.0 * M_PI / ((double)d->n[1] * d->dx[1]);
        p->fk[2] = 2.0 * M_PI / ((double)d->n[2] * d->dx[2]);
        p->dV = d->dx[0] * d->dx[1] * d->dx[2];
    } else {
        g.n0 = d->n[0];
        g.n1 = 1;
        g.nx = d->n[1];
        g.nrows = 1;
        p->fk[0] = 2.0 * M_PI / ((double)d->n[0] * d->dx[0]);
        p->fk[1] = 0.0;
        p->fk[2] = 2.0 * M_PI / ((double)d->n[1] * d->dx[1]);
        p->dV = d->dx[0] * d->dx[1];
    }
    g.M = g.nx / 2;
    g.xrows = g.n0 * g.nrows;
    int64_t Lt = g.nx;
    if (g.n0 > Lt) Lt = g.n0;
    if (g.n1 > Lt) Lt = g.n1;
    g.lt_shift = 0;
    while ((int64_t(1) << g.lt_shift) < Lt) ++g.lt_shift;
    const size_t cs = cx_size(p);
    p->n_partials = (size_t)std::max<int64_t>(2 * pfc::kReduceBlocks, g.xrows);
    // Layout of the packed spectra (Pack in types.hpp), 3D only: rows longer than one 128-byte line
    // padded to whole lines, so that every column tile of the strided passes is line-aligned; and
    // blocks of Z consecutive z planes interleaved by line, so that the z pass reads Z lines in a
    // row per element group.  Whole steps measured on MI355X against plain rows (x rows in natural
    // order): 512^3 FP32 Z = 2 -2.0 %, Z = 4 -1.2 %, Z = 8 +2.2 %; 512^3 FP64 Z = 2 -7.1 %, Z = 4
    // -6.3 %; 2048^3 FP32 Z = 2 -7.5 %, Z = 4 -5.1 %, Z = 8 -6.3 % (larger blocks help the z pass
    // more and stretch the y pass's row stride more).  Z needs a power-of-two z length of at least
    // 256, whose schedules all step by multiples of 8 elements.
    g.Mp = g.M;
    g.zs = 0;
    g.cs = 0;
    if (d->ndim == 3) {
        const int64_t CB = 128 / (int64_t)cs;
        g.cs = (CB == 16) ? 4 : 3;
        if (g.M > CB && g.M % CB != 0) g.Mp = (g.M + CB - 1) / CB * CB;
        const int64_t plane = g.nrows * g.Mp * (int64_t)cs;
        const bool blockable = is_pow2(g.n0) && g.n0 >= 256 && g.Mp % CB == 0;
        if (blockable && plane >= (int64_t(1) << 20)) g.zs = 1;
        // other z lengths take blocks on request where their last-axis schedules step by whole blocks
        auto blocks_ok = [&](int zs) {
            if (blockable) return true;
            if (is_pow2(g.n0) || g.Mp % CB != 0 || g.n0 % (int64_t(1) << zs) != 0) return false;
            return (d->dtype == PFC_F64) ? pfc::z_blocks_ok<double>(g, zs) : pfc::z_blocks_ok<float>(g, zs);
        };
        if (d->flags & 0x10u) {  // PFC_FLAG_ZBLOCK(s): forced block size
            const int zs = (int)((d->flags >> 5) & 3u);
            if (zs > 0 && !blocks_ok(zs)) {
                delete p;
                return fail(PFC_ERR_INVALID_ARG, "PFC_FLAG_ZBLOCK(%d) needs rows of whole 128-byte lines and a z length "
                            "that is a power of two >= 256 or whose last-axis schedules step by whole blocks", zs);
            }
            g.zs = zs;
        }
        g.xnat = (d->flags & PFC_FLAG_XROWS_BLOCK) ? 0 : 1;
    }
    g.nt = state_bytes(p) >= kNonTemporalBytes;
    // after the power-of-two tables: one own table per distinct non-power-of-two pass length
    size_t tw_entries = twiddle_count(Lt);
    std::vector<std::pair<int64_t, int64_t>> mixed;  // (length, entry offset)
    auto table_of = [&](int64_t L) -> int64_t {
        if (!pfc::mixed_length(L)) return 0;
        for (auto &m : mixed)
            if (m.first == L) return m.second;
        mixed.emplace_back(L, (int64_t)tw_entries);
        tw_entries += mix_table_entries(L);
        return mixed.back().second;
    };
    g.tw_x = table_of(g.M);
    g.tw_y = (d->ndim == 3) ? table_of(g.n1) : 0;
    g.tw_last = table_of(g.n0);
    p->tw_entries = tw_entries;
    p->x_fused = (d->dtype == PFC_F64) ? pfc::x_fused_ok<double>(g) : pfc::x_fused_ok<float>(g);
    p->tw_off = 0;
    p->partial_off = align256(tw_entries * cs);
    p->watch_off = p->partial_off + align256(p->n_partials * sizeof(double));
    p->scratch_off = p->watch_off + 256;
    p->ws_need = p->scratch_off + align256(state_bytes(p));
    *out = p;
    return PFC_OK;
}

size_t pfc_plan_workspace_bytes(const pfc_plan *p) { return p ? p->ws_need : 0; }
size_t pfc_plan_real_bytes(const pfc_plan *p) { return p ? real_bytes(p) : 0; }
size_t pfc_plan_half_bytes(const pfc_plan *p) { return p ? half_bytes(p) : 0; }
size_t pfc_plan_state_bytes(const pfc_plan *p) { return p ? state_bytes(p) : 0; }
int pfc_plan_x_fused(const pfc_plan *p)
{
    return (p && p->x_fused && p->var[0] == 0 && p->var[step_passes(p) - 1] == 0) ? 1 : 0;
}

pfc_status pfc_plan_set_workspace(pfc_plan *p, void *dev_ptr, size_t bytes)
{
    if (!p) return fail(PFC_ERR_INVALID_ARG, "plan is NULL");
    if (!dev_ptr) return fail(PFC_ERR_INVALID_ARG, "workspace is NULL");
    if (((uintptr_t)dev_ptr & 255u) != 0) return fail(PFC_ERR_ALIGNMENT, "workspace must be 256-byte aligned");
    if (bytes < p->ws_need) return fail(PFC_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", bytes, p->ws_need);
    const std::vector<char> &host = host_tables(p);
    DeviceGuard dg(p->d.device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
    hipError_t e = hipMemcpy((char *)dev_ptr + p->tw_off, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "twiddle upload");
    p->ws = (char *)dev_ptr;
    p->ws_bytes = bytes;
    return PFC_OK;
}

pfc_status pfc_plan_set_params(pfc_plan *p, double r, double dt)
{
    if (!p) return fail(PFC_ERR_INVALID_ARG, "plan is NULL");
    pfc_plan_desc d = p->d;
    d.r = r;
    d.dt = dt;
    pfc_status st = validate_desc(&d);
    if (st) return st;
    p->d = d;
    return PFC_OK;
}

pfc_status pfc_plan_destroy(pfc_plan *p)
{
    delete p;
    return PFC_OK;
}

#define PFC_DISPATCH(p, fn, ...)                                                   \
    do {                                                                           \
        DeviceGuard dg_((p)->d.device);                                            \
        if (dg_.err != hipSuccess) return hip_fail(dg_.err, "hipSetDevice");       \
        return (p)->d.dtype == PFC_F64 ? fn<double>(__VA_ARGS__) : fn<float>(__VA_ARGS__); \
    } while (0)

#define PFC_CHECK(expr)              \
    do {                             \
        pfc_status st_ = (expr);     \
        if (st_ != PFC_OK) return st_; \
    } while (0)

pfc_status pfc_fft_r2c(pfc_plan *p, const void *real_in, void *half_out, void *stream)
{
    PFC_CHECK(check_ready(p));
    PFC_CHECK(check_ptr(real_in, "real_in"));
    PFC_CHECK(check_ptr(half_out, "half_out"));
    if (overlap(real_in, real_bytes(p), half_out, half_bytes(p)))
        return fail(PFC_ERR_INVALID_ARG, "real_in and half_out overlap");
    PFC_DISPATCH(p, do_r2c, p, real_in, half_out, (hipStream_t)stream);
}

pfc_status pfc_fft_c2r(pfc_plan *p, const void *half_in, void *real_out, void *stream)
{
    PFC_CHECK(check_ready(p));
    PFC_CHECK(check_ptr(half_in, "half_in"));
    PFC_CHECK(check_ptr(real_out, "real_out"));
    if (overlap(half_in, half_bytes(p), real_out, real_bytes(p)))
        return fail(PFC_ERR_INVALID_ARG, "half_in and real_out overlap");
    PFC_DISPATCH(p, do_c2r, p, half_in, real_out, (hipStream_t)stream);
}

pfc_status pfc_state_init(pfc_plan *p, const void *psi0, void *state, void *stream)
{
    PFC_CHECK(check_ready(p));
    PFC_CHECK(check_ptr(psi0, "psi0"));
    PFC_CHECK(check_ptr(state, "state"));
    if (overlap(psi0, real_bytes(p), state, state_bytes(p))) return fail(PFC_ERR_INVALID_ARG, "psi0 and state overlap");
    PFC_DISPATCH(p, do_state_init, p, psi0, state, (hipStream_t)stream);
}

pfc_status pfc_state_export(pfc_plan *p, const void *state, void *half_natural, void *stream)
{
    PFC_CHECK(check_ready(p));
    PFC_CHECK(check_ptr(state, "state"));
    PFC_CHECK(check_ptr(half_natural, "half_natural"));
    if (overlap(state, state_bytes(p), half_natural, half_bytes(p)))
        return fail(PFC_ERR_INVALID_ARG, "state and half_natural overlap");
    PFC_DISPATCH(p, do_export, p, state, half_natural, (hipStream_t)stream);
}

pfc_status pfc_step(pfc_plan *p, void *psi, void *state, int64_t nsteps, void *stream)
{
    PFC_CHECK(check_ready(p));
    PFC_CHECK(check_ptr(psi, "psi"));
    PFC_CHECK(check_ptr(state, "state"));
    if (nsteps < 0) return fail(PFC_ERR_INVALID_ARG, "nsteps < 0");
    if (overlap(psi, real_bytes(p), state, state_bytes(p))) return fail(PFC_ERR_INVALID_ARG, "psi and state overlap");
    PFC_DISPATCH(p, do_step, p, psi, state, nsteps, (hipStream_t)stream);
}

pfc_status pfc_step_watched(pfc_plan *p, void *psi, void *state, int64_t nsteps, int64_t check_every, void *stream,
                            int64_t *done_steps)
{
    PFC_CHECK(check_ready(p));
    PFC_CHECK(check_ptr(psi, "psi"));
    PFC_CHECK(check_ptr(state, "state"));
    if (nsteps < 0 || check_every < 1) return fail(PFC_ERR_INVALID_ARG, "nsteps < 0 or check_every < 1");
    if (!done_steps) return fail(PFC_ERR_INVALID_ARG, "done_steps is NULL");
    if (overlap(psi, real_bytes(p), state, state_bytes(p))) return fail(PFC_ERR_INVALID_ARG, "psi and state overlap");
    PFC_DISPATCH(p, do_step_watched, p, psi, state, nsteps, check_every, (hipStream_t)stream, done_steps);
}

pfc_status pfc_step_timed(pfc_plan *p, void *psi, void *state, int64_t nsteps, void *stream, double *pass_ms,
                          int *npasses)
{
    PFC_CHECK(check_ready(p));
    PFC_CHECK(check_ptr(psi, "psi"));
    PFC_CHECK(check_ptr(state, "state"));
    if (!pass_ms || !npasses) return fail(PFC_ERR_INVALID_ARG, "pass_ms or npasses is NULL");
    if (nsteps < 0) return fail(PFC_ERR_INVALID_ARG, "nsteps < 0");
    if (overlap(psi, real_bytes(p), state, state_bytes(p))) return fail(PFC_ERR_INVALID_ARG, "psi and state overlap");
    *npasses = step_passes(p);
    PFC_DISPATCH(p, do_step_timed, p, psi, state, nsteps, (hipStream_t)stream, pass_ms);
}

pfc_status pfc_plan_autotune(pfc_plan *p, void *psi_scratch, void *state_scratch, void *stream, int reps,
                             double *best_ms)
{
    PFC_CHECK(check_ready(p));
    PFC_CHECK(check_ptr(psi_scratch, "psi_scratch"));
    PFC_CHECK(check_ptr(state_scratch, "state_scratch"));
    if (reps < 1) return fail(PFC_ERR_INVALID_ARG, "reps must be >= 1");
    if (overlap(psi_scratch, real_bytes(p), state_scratch, state_bytes(p)))
        return fail(PFC_ERR_INVALID_ARG, "psi_scratch and state_scratch overlap");
    PFC_DISPATCH(p, do_autotune, p, psi_scratch, state_scratch, (hipStream_t)stream, reps, best_ms);
}

pfc_status pfc_plan_get_tuning(const pfc_plan *p, int *variants, int *npasses)
{
    if (!p || !variants || !npasses) return fail(PFC_ERR_INVALID_ARG, "NULL argument");
    *npasses = step_passes(p);
    for (int k = 0; k < *npasses; ++k) variants[k] = p->var[k];
    return PFC_OK;
}

pfc_status pfc_plan_set_tuning(pfc_plan *p, const int *variants, int npasses)
{
    if (!p || !variants) return fail(PFC_ERR_INVALID_ARG, "NULL argument");
    if (npasses != step_passes(p)) return fail(PFC_ERR_INVALID_ARG, "expected %d passes", step_passes(p));
    for (int k = 0; k < npasses; ++k) {
        const int nc = pfc::step_candidates(p->g, k);
        if (variants[k] < 0 || variants[k] >= nc)
            return fail(PFC_ERR_INVALID_ARG, "pass %d: variant %d out of [0, %d)", k, variants[k], nc);
    }
    for (int k = 0; k < npasses; ++k) p->var[k] = variants[k];
    return PFC_OK;
}

pfc_status pfc_step_backward(pfc_plan *p, const void *psi_n, const void *psi_np1, const void *lambda_np1,
                             void *lambda_n, double *dLdr_accum_dev, void *stream)
{
    PFC_CHECK(check_ready(p));
    PFC_CHECK(check_ptr(psi_n, "psi_n"));
    PFC_CHECK(check_ptr(psi_np1, "psi_np1"));
    PFC_CHECK(check_ptr(lambda_np1, "lambda_np1"));
    PFC_CHECK(check_ptr(lambda_n, "lambda_n"));
    if (!dLdr_accum_dev) return fail(PFC_ERR_INVALID_ARG, "dLdr_accum_dev is NULL");
    const size_t rb = real_bytes(p);
    if (overlap(lambda_n, rb, psi_n, rb) || overlap(lambda_n, rb, psi_np1, rb))
        return fail(PFC_ERR_INVALID_ARG, "lambda_n overlaps psi_n or psi_np1");
    if (lambda_n != lambda_np1 && overlap(lambda_n, rb, lambda_np1, rb))
        return fail(PFC_ERR_INVALID_ARG, "lambda_n partially overlaps lambda_np1");
    PFC_DISPATCH(p, do_backward, p, psi_n, psi_np1, lambda_np1, lambda_n, dLdr_accum_dev, (hipStream_t)stream);
}

size_t pfc_hydro_work_bytes(const pfc_plan *p) { return p ? hydro_work_bytes(p) : 0; }

pfc_status pfc_hydro_state_init(pfc_plan *p, const void *psi, void *psi_state, const void *v, void *v_state,
                                void *stream)
{
    PFC_CHECK(check_ready(p));
    PFC_CHECK(check_ptr(psi, "psi"));
    PFC_CHECK(check_ptr(psi_state, "psi_state"));
    PFC_CHECK(check_ptr(v, "v"));
    PFC_CHECK(check_ptr(v_state, "v_state"));
    PFC_DISPATCH(p, do_hydro_state_init, p, psi, psi_state, v, v_state, (hipStream_t)stream);
}

pfc_status pfc_hydro_step(pfc_plan *p, const pfc_hydro_params *hp, void *psi, void *psi_state, void *v,
                          void *v_state, void *work, size_t work_bytes, int64_t nsteps, void *stream)
{
    PFC_CHECK(check_ready(p));
    if (!hp) return fail(PFC_ERR_INVALID_ARG, "hydro parameters are NULL");
    if (!(hp->rho0 > 0.0) || !std::isfinite(hp->rho0)) return fail(PFC_ERR_INVALID_ARG, "rho0 must be > 0 and finite");
    if (!(hp->gamma >= 0.0) || !std::isfinite(hp->gamma)) return fail(PFC_ERR_INVALID_ARG, "gamma must be >= 0");
    if (!(hp->a0 >= 0.0) || !std::isfinite(hp->a0)) return fail(PFC_ERR_INVALID_ARG, "a0 must be >= 0");
    if (nsteps < 0) return fail(PFC_ERR_INVALID_ARG, "nsteps < 0");
    PFC_CHECK(check_ptr(psi, "psi"));
    PFC_CHECK(check_ptr(psi_state, "psi_state"));
    PFC_CHECK(check_ptr(v, "v"));
    PFC_CHECK(check_ptr(v_state, "v_state"));
    if (!work || work_bytes < hydro_work_bytes(p))
        return fail(PFC_ERR_WORKSPACE, "hydro work buffer has %zu bytes, needs %zu", work ? work_bytes : (size_t)0,
                    hydro_work_bytes(p));
    if (((uintptr_t)work & 255u) != 0) return fail(PFC_ERR_ALIGNMENT, "hydro work buffer must be 256-byte aligned");
    const size_t nd = (size_t)p->g.ndim;
    if (overlap(work, hydro_work_bytes(p), psi, real_bytes(p)) || overlap(work, hydro_work_bytes(p), v, nd * real_bytes(p)) ||
        overlap(work, hydro_work_bytes(p), psi_state, state_bytes(p)) ||
        overlap(work, hydro_work_bytes(p), v_state, nd * state_bytes(p)))
        return fail(PFC_ERR_INVALID_ARG, "hydro work buffer overlaps a field");
    PFC_DISPATCH(p, do_hydro_step, p, hp, psi, psi_state, v, v_state, work, nsteps, (hipStream_t)stream);
}

pfc_status pfc_energy(pfc_plan *p, const void *psi, const void *state, double *out_dev, void *stream)
{
    PFC_CHECK(check_ready(p));
    PFC_CHECK(check_ptr(psi, "psi"));
    PFC_CHECK(check_ptr(state, "state"));
    if (!out_dev) return fail(PFC_ERR_INVALID_ARG, "out_dev is NULL");
    PFC_DISPATCH(p, do_energy, p, psi, state, out_dev, (hipStream_t)stream);
}

pfc_status pfc_batch_create(pfc_batch **out, const pfc_plan_desc *descs, int count)
{
    if (!out) return fail(PFC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!descs || count < 1 || count > pfc::kBatchMaxInstHost)
        return fail(PFC_ERR_INVALID_ARG, "count must be in [1, %d]", pfc::kBatchMaxInstHost);
    for (int i = 0; i < count; ++i) {
        const pfc_plan_desc &d = descs[i];
        if (d.ndim != 2) return fail(PFC_ERR_UNSUPPORTED, "instance %d: the batched form takes 2D grids", i);
        for (int a = 0; a < 2; ++a)
            if (!is_pow2(d.n[a]) || d.n[a] < 32 || d.n[a] > 1024)
                return fail(PFC_ERR_UNSUPPORTED, "instance %d: n[%d] = %lld, batched sizes are powers of two in "
                            "[32, 1024]", i, a, (long long)d.n[a]);
        pfc_status st = validate_desc(&d);
        if (st) return fail(st, "instance %d: %s", i, g_last_error.c_str());
        if (d.dtype != descs[0].dtype) return fail(PFC_ERR_INVALID_ARG, "instance %d: dtypes differ", i);
        if (d.device != descs[0].device) return fail(PFC_ERR_INVALID_ARG, "instance %d: devices differ", i);
    }
    pfc_batch *b = new (std::nothrow) pfc_batch();
    if (!b) return fail(PFC_ERR_INTERNAL, "out of host memory");
    b->count = count;
    b->dtype = descs[0].dtype;
    b->device = descs[0].device;
    b->descs.assign(descs, descs + count);
    int64_t Lt = 4;
    for (int i = 0; i < count; ++i) {
        pfc_batch::Inst g;
        g.n0 = (int)descs[i].n[0];
        g.nx = (int)descs[i].n[1];
        g.M = g.nx / 2;
        b->inst.push_back(g);
        Lt = std::max<int64_t>(Lt, std::max(g.n0, g.nx));
    }
    {
        pfc_status st = batch_layout(b);
        if (st) {
            delete b;
            return st;
        }
    }
    while ((int64_t(1) << b->lt_shift) < Lt) ++b->lt_shift;
    // largest instances first: their items are the longest, so they start first
    b->order.resize(count);
    std::iota(b->order.begin(), b->order.end(), 0);
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) {
        return (int64_t)b->inst[x].n0 * b->inst[x].nx > (int64_t)b->inst[y].n0 * b->inst[y].nx;
    });
    const size_t cs = b->dtype == PFC_F64 ? 16 : 8;
    const size_t inst_size = b->dtype == PFC_F64 ? sizeof(pfc::BatchInst<double>) : sizeof(pfc::BatchInst<float>);
    b->ctl_off = 0;
    b->inst_off = 256;
    b->tw_off = b->inst_off + align256(inst_size * count);
    b->partial_off = b->tw_off + align256(twiddle_count(Lt) * cs);
    size_t off = b->partial_off + align256(pfc::kReduceBlocks * sizeof(double));
    for (int i = 0; i < count; ++i) {
        b->scratch_off.push_back(off);
        off += align256((size_t)b->inst[i].n0 * b->inst[i].M * cs);
    }
    b->ws_need = off;
    *out = b;
    return PFC_OK;
}

size_t pfc_batch_workspace_bytes(const pfc_batch *b) { return b ? b->ws_need : 0; }

int pfc_batch_grid(const pfc_batch *b) { return b ? b->grid : 0; }

pfc_status pfc_batch_bind(pfc_batch *b, void *const *psi, void *const *state, void *workspace, size_t bytes)
{
    if (!b) return fail(PFC_ERR_INVALID_ARG, "batch is NULL");
    if (!psi || !state) return fail(PFC_ERR_INVALID_ARG, "psi or state array is NULL");
    if (!workspace) return fail(PFC_ERR_INVALID_ARG, "workspace is NULL");
    if (((uintptr_t)workspace & 255u) != 0) return fail(PFC_ERR_ALIGNMENT, "workspace must be 256-byte aligned");
    if (bytes < b->ws_need) return fail(PFC_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", bytes, b->ws_need);
    const size_t cs = b->dtype == PFC_F64 ? 16 : 8;
    for (int i = 0; i < b->count; ++i) {
        PFC_CHECK(check_ptr(psi[i], "psi[i]"));
        PFC_CHECK(check_ptr(state[i], "state[i]"));
        const size_t n = (size_t)b->inst[i].n0 * b->inst[i].M * cs;
        if (overlap(psi[i], n, state[i], n)) return fail(PFC_ERR_INVALID_ARG, "psi[%d] and state[%d] overlap", i, i);
        if (overlap(psi[i], n, workspace, bytes) || overlap(state[i], n, workspace, bytes))
            return fail(PFC_ERR_INVALID_ARG, "instance %d overlaps the workspace", i);
    }
    DeviceGuard dg(b->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
    drop_graphs(b);
    b->psi.assign(psi, psi + b->count);
    b->state.assign(state, state + b->count);
    b->ws = (char *)workspace;
    b->ws_bytes = bytes;
    pfc_status st = b->dtype == PFC_F64 ? batch_bind_impl<double>(b) : batch_bind_impl<float>(b);
    if (st) b->ws = nullptr;
    return st;
}

pfc_status pfc_batch_state_init(pfc_batch *b, void *stream)
{
    if (!b || !b->ws) return fail(PFC_ERR_WORKSPACE, "batch not bound");
    DeviceGuard dg(b->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
    return b->dtype == PFC_F64 ? batch_state_init_impl<double>(b, (hipStream_t)stream)
                               : batch_state_init_impl<float>(b, (hipStream_t)stream);
}

pfc_status pfc_batch_step(pfc_batch *b, int64_t nsteps, void *stream)
{
    if (!b || !b->ws) return fail(PFC_ERR_WORKSPACE, "batch not bound");
    if (nsteps < 0) return fail(PFC_ERR_INVALID_ARG, "nsteps < 0");
    if (nsteps == 0) return PFC_OK;
    DeviceGuard dg(b->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
    return b->dtype == PFC_F64 ? batch_step_impl<double>(b, nsteps, (hipStream_t)stream)
                               : batch_step_impl<float>(b, nsteps, (hipStream_t)stream);
}

pfc_status pfc_batch_check(pfc_batch *b, void *stream)
{
    if (!b || !b->ws) return fail(PFC_ERR_WORKSPACE, "batch not bound");
    DeviceGuard dg(b->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
    PFC_TRY(hipStreamSynchronize((hipStream_t)stream), "stream synchronize");
    pfc::BatchCtl ctl;
    PFC_TRY(hipMemcpy(&ctl, b->ws + b->ctl_off, sizeof ctl, hipMemcpyDeviceToHost), "barrier state read");
    if (ctl.err) {
        PFC_TRY(hipMemset(b->ws + b->ctl_off, 0, sizeof ctl), "barrier state reset");
        return fail(PFC_ERR_INTERNAL, "a grid barrier of the batched kernel timed out (workgroups not all resident); "
                    "results of that launch are incomplete");
    }
    return PFC_OK;
}

pfc_status pfc_batch_get_tuning(const pfc_batch *b, int *variants, int n)
{
    if (!b || !variants) return fail(PFC_ERR_INVALID_ARG, "NULL argument");
    if (n != 3 * b->count) return fail(PFC_ERR_INVALID_ARG, "expected %d entries (3 per instance)", 3 * b->count);
    for (int i = 0; i < b->count; ++i) {
        variants[3 * i] = b->inst[i].vx;
        variants[3 * i + 1] = b->inst[i].vy;
        variants[3 * i + 2] = b->inst[i].vc;
    }
    return PFC_OK;
}

pfc_status pfc_batch_set_tuning(pfc_batch *b, const int *variants, int n)
{
    if (!b || !variants) return fail(PFC_ERR_INVALID_ARG, "NULL argument");
    if (n != 3 * b->count) return fail(PFC_ERR_INVALID_ARG, "expected %d entries (3 per instance)", 3 * b->count);
    for (int i = 0; i < b->count; ++i)
        for (int k = 0; k < 3; ++k) {
            const int nc = pfc::batch_candidates(b->inst[i].n0, b->inst[i].M, k);
            if (variants[3 * i + k] < 0 || variants[3 * i + k] >= nc)
                return fail(PFC_ERR_INVALID_ARG, "instance %d pass %d: variant %d out of [0, %d)", i, k,
                            variants[3 * i + k], nc);
        }
    std::vector<pfc_batch::Inst> saved = b->inst;
    for (int i = 0; i < b->count; ++i) {
        b->inst[i].vx = variants[3 * i];
        b->inst[i].vy = variants[3 * i + 1];
        b->inst[i].vc = variants[3 * i + 2];
    }
    pfc_status st = batch_layout(b);
    if (st) {
        b->inst = saved;
        return st;
    }
    if (!b->ws) return PFC_OK;
    DeviceGuard dg(b->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
    return b->dtype == PFC_F64 ? batch_upload_table<double>(b) : batch_upload_table<float>(b);
}

pfc_status pfc_batch_autotune(pfc_batch *b, void *stream, int steps, double *ms_per_step)
{
    if (!b || !b->ws) return fail(PFC_ERR_WORKSPACE, "batch not bound");
    if (steps < 1) return fail(PFC_ERR_INVALID_ARG, "steps must be >= 1");
    DeviceGuard dg(b->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
    return b->dtype == PFC_F64 ? batch_autotune_impl<double>(b, (hipStream_t)stream, steps, ms_per_step)
                               : batch_autotune_impl<float>(b, (hipStream_t)stream, steps, ms_per_step);
}

pfc_status pfc_batch_destroy(pfc_batch *b)
{
    if (!b) return PFC_OK;
    drop_graphs(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return PFC_OK;
}

const char *pfc_status_string(pfc_status st)
{
    switch (st) {
    case PFC_OK: return "PFC_OK";
    case PFC_ERR_INVALID_ARG: return "PFC_ERR_INVALID_ARG";
    case PFC_ERR_UNSUPPORTED: return "PFC_ERR_UNSUPPORTED";
    case PFC_ERR_ALIGNMENT: return "PFC_ERR_ALIGNMENT";
    case PFC_ERR_WORKSPACE: return "PFC_ERR_WORKSPACE";
    case PFC_ERR_HIP: return "PFC_ERR_HIP";
    case PFC_ERR_DIVERGED: return "PFC_ERR_DIVERGED";
    case PFC_ERR_INTERNAL: return "PFC_ERR_INTERNAL";
    }
    return "unknown pfc_status";
}

const char *pfc_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

// ------------------------------------------------------------------------------------------------
// Complex-amplitude form (contract in include/pfc.h; kernels in apfc.hpp).

struct pfc_apfc {
    pfc_apfc_desc d;
    int64_t n0, n1, nx, P;  // 2D: n1 = 1
    double fk[3];           // 2 pi / (n dx) along (axis 0, axis 1, x)
    int lt_shift = 0;
    bool nt = false;
    int64_t tw_x = 0, tw_y = 0, tw_last = 0;
    size_t tw_entries = 0;
    std::vector<pfc::ApfcTerm> terms;
    std::vector<int> off;   // terms of field j: [off[j], off[j+1])
    std::vector<int> npairs, ntriples;
    size_t tw_off = 0, terms_off = 0, off_off = 0, scratch_off = 0, ws_need = 0;
    char *ws = nullptr;
};

namespace {

size_t apfc_cx(const pfc_apfc *p) { return p->d.dtype == PFC_F64 ? 16 : 8; }
size_t apfc_field_bytes(const pfc_apfc *p) { return (size_t)p->P * (size_t)p->d.nfields * apfc_cx(p); }

bool apfc_length_ok(int64_t n) { return (is_pow2(n) && n >= 4 && n <= 2048) || (pfc::mixed_length(n) && n % 2 == 0); }

// Resonant products of every amplitude.  Signed index s = +-(f+1); k_{-a} = -k_a.  Ordered tuples
// whose vector sum is within tol of k_j are counted per unordered product, and the count becomes
// the product's multiplicity.
void apfc_products(pfc_apfc *p)
{
    const pfc_apfc_desc &d = p->d;
    const int N = d.nfields, nd = d.ndim;
    double kmax = 0.0;
    for (int j = 0; j < N; ++j) {
        double kk = 0.0;
        for (int a = 0; a < nd; ++a) kk += d.k[j][a] * d.k[j][a];
        kmax = std::max(kmax, std::sqrt(kk));
    }
    const double tol = 1e-9 * kmax;
    std::vector<int> sig;
    for (int f = 1; f <= N; ++f) {
        sig.push_back(f);
        sig.push_back(-f);
    }
    auto comp = [&](int s, int a) { return s > 0 ? d.k[s - 1][a] : -d.k[-s - 1][a]; };
    p->terms.clear();
    p->off.assign(1, 0);
    p->npairs.clear();
    p->ntriples.clear();
    for (int j = 0; j < N; ++j) {
        auto hits = [&](const int *s, int len) {
            for (int a = 0; a < nd; ++a) {
                double sum = 0.0;
                for (int i = 0; i < len; ++i) sum += comp(s[i], a);
                if (std::fabs(sum - d.k[j][a]) > tol) return false;
            }
            return true;
        };
        std::map<std::vector<int>, int> pairs, triples;
        for (int x : sig)
            for (int y : sig) {
                const int s2[2] = {x, y};
                if (hits(s2, 2)) {
                    std::vector<int> key(s2, s2 + 2);
                    std::sort(key.begin(), key.end());
                    ++pairs[key];
                }
                for (int z : sig) {
                    const int s3[3] = {x, y, z};
                    if (hits(s3, 3)) {
                        std::vector<int> key(s3, s3 + 3);
                        std::sort(key.begin(), key.end());
                        ++triples[key];
                    }
                }
            }
        // the permutations of (j, i, -i) are evaluated in closed form by the kernel (3 orders for
        // i = j, 6 otherwise: every one of them is resonant, so none is left over)
        for (int i = 1; i <= N; ++i) {
            std::vector<int> key = {j + 1, i, -i};
            std::sort(key.begin(), key.end());
            triples.erase(key);
        }
        int np = 0, nt = 0;
        if (d.t != 0.0)
            for (auto &kv : pairs) {
                pfc::ApfcTerm m{};
                m.a = (int16_t)kv.first[0];
                m.b = (int16_t)kv.first[1];
                m.c = 0;
                m.coef = -d.t * kv.second;
                m.coef32 = (float)m.coef;
                p->terms.push_back(m);
                ++np;
            }
        if (d.v != 0.0)
            for (auto &kv : triples) {
                pfc::ApfcTerm m{};
                m.a = (int16_t)kv.first[0];
                m.b = (int16_t)kv.first[1];
                m.c = (int16_t)kv.first[2];
                m.coef = d.v * kv.second;
                m.coef32 = (float)m.coef;
                p->terms.push_back(m);
                ++nt;
            }
        p->npairs.push_back(np);
        p->ntriples.push_back(nt);
        p->off.push_back((int)p->terms.size());
    }
}

pfc_status apfc_validate(const pfc_apfc_desc *d)
{
    if (d->ndim != 2 && d->ndim != 3) return fail(PFC_ERR_INVALID_ARG, "ndim must be 2 or 3");
    if (d->dtype != PFC_F32 && d->dtype != PFC_F64) return fail(PFC_ERR_INVALID_ARG, "bad dtype");
    for (int a = 0; a < d->ndim; ++a) {
        if (!apfc_length_ok(d->n[a]))
            return fail(PFC_ERR_UNSUPPORTED, "axis %d: length %lld has no compiled schedule", a, (long long)d->n[a]);
        if (!(d->dx[a] > 0.0) || !std::isfinite(d->dx[a])) return fail(PFC_ERR_INVALID_ARG, "dx[%d] must be > 0", a);
    }
    if (d->nfields < 1 || d->nfields > PFC_APFC_MAX_FIELDS)
        return fail(PFC_ERR_INVALID_ARG, "nfields must be in [1, %d]", PFC_APFC_MAX_FIELDS);
    if (!(d->dt > 0.0) || !std::isfinite(d->dt)) return fail(PFC_ERR_INVALID_ARG, "dt must be > 0");
    if (!(d->Bx >= 0.0) || !std::isfinite(d->Bx)) return fail(PFC_ERR_INVALID_ARG, "Bx must be >= 0");
    if (!std::isfinite(d->dB) || !std::isfinite(d->t) || !std::isfinite(d->v))
        return fail(PFC_ERR_INVALID_ARG, "dB, t, v must be finite");
    for (int j = 0; j < d->nfields; ++j) {
        double kk = 0.0;
        for (int a = 0; a < d->ndim; ++a) {
            if (!std::isfinite(d->k[j][a])) return fail(PFC_ERR_INVALID_ARG, "k[%d] is not finite", j);
            kk += d->k[j][a] * d->k[j][a];
        }
        if (!(kk > 0.0)) return fail(PFC_ERR_INVALID_ARG, "k[%d] is zero", j);
        // the denominator 1 + dt |k|^2 (dB + Bx G^2) is smallest at G = 0 (Bx >= 0)
        if (!(1.0 + d->dt * kk * d->dB > 0.0))
            return fail(PFC_ERR_INVALID_ARG, "1 + dt |k_%d|^2 dB <= 0: dt too large for this dB", j);
    }
    return PFC_OK;
}

pfc_status apfc_ready(const pfc_apfc *p)
{
    if (!p) return fail(PFC_ERR_INVALID_ARG, "object is NULL");
    if (!p->ws) return fail(PFC_ERR_WORKSPACE, "no workspace attached (pfc_apfc_set_workspace)");
    return PFC_OK;
}

// the y pass and the FFT-only last-axis pass reuse the PFC pencil launchers through a geometry
// that treats the fields as extra planes
pfc::Geom apfc_y_geom(const pfc_apfc *p)
{
    pfc::Geom g{};
    g.ndim = 3;
    g.n0 = (int64_t)p->d.nfields * p->n0;
    g.n1 = p->n1;
    g.nx = p->nx;
    g.M = p->nx;
    g.nrows = p->n1;
    g.xrows = g.n0 * g.nrows;
    g.lt_shift = p->lt_shift;
    g.nt = p->nt;
    g.tw_y = p->tw_y;
    return g;
}
pfc::Geom apfc_last_geom(const pfc_apfc *p)
{
    pfc::Geom g{};
    g.ndim = p->d.ndim;
    g.n0 = p->n0;
    g.n1 = p->n1;
    g.nx = p->nx;
    g.M = p->nx;
    g.nrows = p->n1;
    g.xrows = g.n0 * g.nrows;
    g.lt_shift = p->lt_shift;
    g.tw_last = p->tw_last;
    return g;
}

template <typename T>
const cx<T> *apfc_tw(const pfc_apfc *p)
{
    return reinterpret_cast<const cx<T> *>(p->ws + p->tw_off);
}

template <typename T>
pfc_status do_apfc_fft(pfc_apfc *p, const void *in_v, void *out_v, int dir, hipStream_t s)
{
    const cx<T> *in = (const cx<T> *)in_v;
    cx<T> *out = (cx<T> *)out_v;
    const cx<T> *tw = apfc_tw<T>(p);
    const int N = p->d.nfields;
    const int64_t rows = (int64_t)N * p->n0 * p->n1;
    const pfc::Geom gy = apfc_y_geom(p), gl = apfc_last_geom(p);
    if (dir < 0) {
        PFC_TRY(pfc::launch_apfc_rows<T>(p->nx, in, out, rows, -1, 1.0, p->nt, tw + p->tw_x, p->lt_shift, s),
                "x forward launch");
        if (p->d.ndim == 3) PFC_TRY(pfc::launch_y_c2c<T>(gy, out, -1, tw, s), "y forward launch");
        for (int f = 0; f < N; ++f)
            PFC_TRY(pfc::launch_last_c2c<T>(gl, out + f * p->P, out + f * p->P, -1, tw, s), "last-axis forward launch");
    } else {
        for (int f = 0; f < N; ++f)
            PFC_TRY(pfc::launch_last_c2c<T>(gl, in + f * p->P, out + f * p->P, +1, tw, s), "last-axis inverse launch");
        if (p->d.ndim == 3) PFC_TRY(pfc::launch_y_c2c<T>(gy, out, +1, tw, s), "y inverse launch");
        PFC_TRY(pfc::launch_apfc_rows<T>(p->nx, out, out, rows, +1, 1.0 / (double)p->P, p->nt, tw + p->tw_x,
                                         p->lt_shift, s),
                "x inverse launch");
    }
    return PFC_OK;
}

template <typename T>
pfc_status do_apfc_nonlinear(pfc_apfc *p, const void *eta, void *out, hipStream_t s)
{
    const pfc::ApfcTerm *terms = reinterpret_cast<const pfc::ApfcTerm *>(p->ws + p->terms_off);
    const int *off = reinterpret_cast<const int *>(p->ws + p->off_off);
    PFC_TRY(pfc::launch_apfc_nonlin<T>((const cx<T> *)eta, (cx<T> *)out, p->P, p->d.nfields, terms, off,
                                       3.0 * p->d.v, s),
            "nonlinearity launch");
    return PFC_OK;
}

template <typename T>
pfc_status do_apfc_step(pfc_apfc *p, void *eta_v, void *eta_hat_v, int64_t nsteps, hipStream_t s)
{
    cx<T> *eta = (cx<T> *)eta_v, *S = (cx<T> *)eta_hat_v;
    cx<T> *scr = reinterpret_cast<cx<T> *>(p->ws + p->scratch_off);
    const cx<T> *tw = apfc_tw<T>(p);
    const pfc_apfc_desc &d = p->d;
    const int N = d.nfields;
    const int64_t rows = (int64_t)N * p->n0 * p->n1;
    const pfc::Geom gy = apfc_y_geom(p);
    pfc::ApfcStepArgs<T> a{};
    a.src = scr;
    a.dst = scr;
    a.state = S;
    a.ncols = p->n1 * p->nx;
    a.nx = p->nx;
    a.n1 = p->n1;
    a.fstride = p->P;
    for (int i = 0; i < 3; ++i) a.fk[i] = (T)p->fk[i];
    a.dt = (T)d.dt;
    a.dB = (T)d.dB;
    a.Bx = (T)d.Bx;
    for (int f = 0; f < N; ++f) {
        // components along (axis 0, axis 1, x); axis 1 is absent in 2D
        const double k0 = d.k[f][0], k1 = d.ndim == 3 ? d.k[f][1] : 0.0, kx = d.k[f][d.ndim - 1];
        a.kv[f][0] = (T)k0;
        a.kv[f][1] = (T)k1;
        a.kv[f][2] = (T)kx;
        a.kk[f] = (T)(k0 * k0 + k1 * k1 + kx * kx);
    }
    a.tw = tw + p->tw_last;
    a.lt_shift = p->lt_shift;
    for (int64_t st = 0; st < nsteps; ++st) {
        pfc_status e = do_apfc_nonlinear<T>(p, eta, scr, s);
        if (e) return e;
        PFC_TRY(pfc::launch_apfc_rows<T>(p->nx, scr, scr, rows, -1, 1.0, p->nt, tw + p->tw_x, p->lt_shift, s),
                "x forward launch");
        if (d.ndim == 3) PFC_TRY(pfc::launch_y_c2c<T>(gy, scr, -1, tw, s), "y forward launch");
        PFC_TRY(pfc::launch_apfc_last_step<T>(p->n0, N, a, s), "last-axis step launch");
        if (d.ndim == 3) PFC_TRY(pfc::launch_y_c2c<T>(gy, scr, +1, tw, s), "y inverse launch");
        PFC_TRY(pfc::launch_apfc_rows<T>(p->nx, scr, eta, rows, +1, 1.0 / (double)p->P, p->nt, tw + p->tw_x,
                                         p->lt_shift, s),
                "x inverse launch");
    }
    return PFC_OK;
}

pfc_status apfc_fields(const pfc_apfc *p, const void *a, const char *na, const void *b, const char *nb)
{
    for (auto pr : {std::make_pair(a, na), std::make_pair(b, nb)}) {
        if (!pr.first) return fail(PFC_ERR_INVALID_ARG, "%s is NULL", pr.second);
        if (!aligned16(pr.first)) return fail(PFC_ERR_ALIGNMENT, "%s is not 16-byte aligned", pr.second);
        if (overlap(pr.first, apfc_field_bytes(p), p->ws, p->ws_need))
            return fail(PFC_ERR_INVALID_ARG, "%s overlaps the workspace", pr.second);
    }
    return PFC_OK;
}

}  // namespace

#define PFC_APFC_DISPATCH(p, fn, ...)                                              \
    do {                                                                           \
        DeviceGuard dg_((p)->d.device);                                            \
        if (dg_.err != hipSuccess) return hip_fail(dg_.err, "hipSetDevice");       \
        return (p)->d.dtype == PFC_F64 ? fn<double>(__VA_ARGS__) : fn<float>(__VA_ARGS__); \
    } while (0)

extern "C" {

pfc_status pfc_apfc_create(pfc_apfc **out, const pfc_apfc_desc *d)
{
    if (!out) return fail(PFC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!d) return fail(PFC_ERR_INVALID_ARG, "descriptor is NULL");
    PFC_CHECK(apfc_validate(d));
    pfc_apfc *p = new (std::nothrow) pfc_apfc;
    if (!p) return fail(PFC_ERR_INTERNAL, "out of host memory");
    p->d = *d;
    p->n0 = d->n[0];
    p->n1 = d->ndim == 3 ? d->n[1] : 1;
    p->nx = d->n[d->ndim - 1];
    p->P = p->n0 * p->n1 * p->nx;
    p->fk[0] = 2.0 * M_PI / ((double)d->n[0] * d->dx[0]);
    p->fk[1] = d->ndim == 3 ? 2.0 * M_PI / ((double)d->n[1] * d->dx[1]) : 0.0;
    p->fk[2] = 2.0 * M_PI / ((double)p->nx * d->dx[d->ndim - 1]);
    int64_t Lt = std::max(p->n0, std::max(p->n1, p->nx));
    while ((int64_t(1) << p->lt_shift) < Lt) ++p->lt_shift;
    size_t tw_entries = twiddle_count(int64_t(1) << p->lt_shift);
    std::vector<std::pair<int64_t, int64_t>> mixed;
    auto table_of = [&](int64_t L) -> int64_t {
        if (!pfc::mixed_length(L)) return 0;
        for (auto &m : mixed)
            if (m.first == L) return m.second;
        mixed.emplace_back(L, (int64_t)tw_entries);
        tw_entries += mix_table_entries(L);
        return mixed.back().second;
    };
    p->tw_x = table_of(p->nx);
    p->tw_y = d->ndim == 3 ? table_of(p->n1) : 0;
    p->tw_last = table_of(p->n0);
    p->tw_entries = tw_entries;
    p->nt = apfc_field_bytes(p) >= kNonTemporalBytes;
    apfc_products(p);
    const size_t cs = apfc_cx(p);
    p->tw_off = 0;
    p->terms_off = align256(tw_entries * cs);
    p->off_off = p->terms_off + align256(std::max<size_t>(1, p->terms.size()) * sizeof(pfc::ApfcTerm));
    p->scratch_off = p->off_off + align256(p->off.size() * sizeof(int));
    p->ws_need = p->scratch_off + align256(apfc_field_bytes(p));
    *out = p;
    return PFC_OK;
}

size_t pfc_apfc_field_bytes(const pfc_apfc *p) { return p ? apfc_field_bytes(p) : 0; }
size_t pfc_apfc_workspace_bytes(const pfc_apfc *p) { return p ? p->ws_need : 0; }

pfc_status pfc_apfc_set_workspace(pfc_apfc *p, void *dev_ptr, size_t bytes)
{
    if (!p) return fail(PFC_ERR_INVALID_ARG, "object is NULL");
    if (!dev_ptr) return fail(PFC_ERR_INVALID_ARG, "workspace is NULL");
    if (((uintptr_t)dev_ptr & 255u) != 0) return fail(PFC_ERR_ALIGNMENT, "workspace must be 256-byte aligned");
    if (bytes < p->ws_need) return fail(PFC_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", bytes, p->ws_need);
    std::vector<char> host(p->scratch_off, 0);
    auto build = [&](auto tc) {
        using T = decltype(tc);
        std::vector<cx<T>> tw = twiddle_table<T>(int64_t(1) << p->lt_shift);
        tw.resize(p->tw_entries);
        const int64_t lens[3] = {p->nx, p->d.ndim == 3 ? p->n1 : 0, p->n0};
        const int64_t offs[3] = {p->tw_x, p->tw_y, p->tw_last};
        for (int i = 0; i < 3; ++i)
            if (offs[i] > 0)
                with_mixed_length(lens[i], [&](auto lc) { fill_mix_table<T, decltype(lc)::value>(tw.data() + offs[i]); });
        std::memcpy(host.data() + p->tw_off, tw.data(), tw.size() * sizeof(cx<T>));
    };
    if (p->d.dtype == PFC_F64)
        build(double{});
    else
        build(float{});
    if (!p->terms.empty())
        std::memcpy(host.data() + p->terms_off, p->terms.data(), p->terms.size() * sizeof(pfc::ApfcTerm));
    std::memcpy(host.data() + p->off_off, p->off.data(), p->off.size() * sizeof(int));
    DeviceGuard dg(p->d.device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
    hipError_t e = hipMemcpy(dev_ptr, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "table upload");
    p->ws = (char *)dev_ptr;
    return PFC_OK;
}

pfc_status pfc_apfc_terms(const pfc_apfc *p, int j, int *npairs, int *ntriples)
{
    if (!p) return fail(PFC_ERR_INVALID_ARG, "object is NULL");
    if (j < 0 || j >= p->d.nfields) return fail(PFC_ERR_INVALID_ARG, "field %d out of range", j);
    if (npairs) *npairs = p->npairs[j];
    if (ntriples) *ntriples = p->ntriples[j];
    return PFC_OK;
}

pfc_status pfc_apfc_fft(pfc_apfc *p, const void *in, void *out, int dir, void *stream)
{
    PFC_CHECK(apfc_ready(p));
    if (dir != -1 && dir != 1) return fail(PFC_ERR_INVALID_ARG, "dir must be -1 or +1");
    PFC_CHECK(apfc_fields(p, in, "in", out, "out"));
    if (in != out && overlap(in, apfc_field_bytes(p), out, apfc_field_bytes(p)))
        return fail(PFC_ERR_INVALID_ARG, "in and out overlap without being equal");
    PFC_APFC_DISPATCH(p, do_apfc_fft, p, in, out, dir, (hipStream_t)stream);
}

pfc_status pfc_apfc_nonlinear(pfc_apfc *p, const void *eta, void *out, void *stream)
{
    PFC_CHECK(apfc_ready(p));
    PFC_CHECK(apfc_fields(p, eta, "eta", out, "out"));
    if (overlap(eta, apfc_field_bytes(p), out, apfc_field_bytes(p))) return fail(PFC_ERR_INVALID_ARG, "eta and out overlap");
    PFC_APFC_DISPATCH(p, do_apfc_nonlinear, p, eta, out, (hipStream_t)stream);
}

pfc_status pfc_apfc_state_init(pfc_apfc *p, const void *eta, void *eta_hat, void *stream)
{
    return pfc_apfc_fft(p, eta, eta_hat, -1, stream);
}

pfc_status pfc_apfc_step(pfc_apfc *p, void *eta, void *eta_hat, int64_t nsteps, void *stream)
{
    PFC_CHECK(apfc_ready(p));
    if (nsteps < 0) return fail(PFC_ERR_INVALID_ARG, "nsteps < 0");
    PFC_CHECK(apfc_fields(p, eta, "eta", eta_hat, "eta_hat"));
    if (overlap(eta, apfc_field_bytes(p), eta_hat, apfc_field_bytes(p)))
        return fail(PFC_ERR_INVALID_ARG, "eta and eta_hat overlap");
    PFC_APFC_DISPATCH(p, do_apfc_step, p, eta, eta_hat, nsteps, (hipStream_t)stream);
}

pfc_status pfc_apfc_destroy(pfc_apfc *p)
{
    delete p;
    return PFC_OK;
}

}  // extern "C"

// ---- internal calls of the allocation-free step (api_internal.hpp)
namespace pfc_internal {

size_t table_bytes(const pfc_plan *p) { return align256(p->tw_entries * cx_size(p)); }
size_t spectrum_bytes(const pfc_plan *p) { return state_bytes(p); }
int plan_device(const pfc_plan *p) { return p->d.device; }
uint64_t plan_id(const pfc_plan *p) { return p->id; }
pfc_status report(pfc_status st, const char *msg) { return fail(st, "%s", msg); }

pfc_status check_step_args(const pfc_plan *p, const void *psi, const void *state, int64_t nsteps)
{
    if (!p) return fail(PFC_ERR_INVALID_ARG, "plan is NULL");
    PFC_CHECK(check_ptr(psi, "psi"));
    PFC_CHECK(check_ptr(state, "state"));
    if (nsteps < 0) return fail(PFC_ERR_INVALID_ARG, "nsteps < 0");
    if (overlap(psi, real_bytes(p), state, state_bytes(p))) return fail(PFC_ERR_INVALID_ARG, "psi and state overlap");
    return PFC_OK;
}

pfc_status upload_tables(pfc_plan *p, void *tables, void *stream)
{
    const std::vector<char> &host = host_tables(p);
    PFC_TRY(hipMemcpyAsync(tables, host.data(), host.size(), hipMemcpyHostToDevice, (hipStream_t)stream),
            "twiddle upload");
    return PFC_OK;
}

template <typename T>
static pfc_status step_in(pfc_plan *p, void *psi, void *state, int64_t nsteps, hipStream_t s, void *tables,
                          void *spectrum)
{
    const Bufs<T> b{reinterpret_cast<const cx<T> *>(tables), nullptr, reinterpret_cast<cx<T> *>(spectrum)};
    return step_with<T>(p, b, psi, state, nsteps, s);
}

pfc_status step_with_buffers(pfc_plan *p, void *psi, void *state, int64_t nsteps, void *stream, void *tables,
                             void *spectrum)
{
    return p->d.dtype == PFC_F64 ? step_in<double>(p, psi, state, nsteps, (hipStream_t)stream, tables, spectrum)
                                 : step_in<float>(p, psi, state, nsteps, (hipStream_t)stream, tables, spectrum);
}

}  // namespace pfc_internal
