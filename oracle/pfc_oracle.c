/*
 * pfc_oracle.c -- plain FP64 CPU oracle for the pseudo-spectral phase-field-crystal (PFC) step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this library.  It shares no code, header, table or helper with the HIP library.
 *
 * What it computes (arxiv 2603.26818, "Multi-GPU fast Fourier transforms in MATLAB for large-scale
 * phase-field crystal simulations"):
 *   - the discrete Fourier transform used by the Fourier pseudo-spectral method (section "Fourier
 *     pseudo-spectral method", Eq. (2) and the paragraph after it): forward e^{-ikx} unnormalised,
 *     inverse with 1/N, computed by a textbook recursive Cooley-Tukey FFT (decimation in time over
 *     the smallest prime factor of the length: radix 2 for powers of two, a plain p-point DFT per
 *     output group otherwise) applied row-column along every axis;
 *   - the PFC free energy, Eq. (3), and the PFC dynamics, Eq. (4), with the correlation operator
 *     written as a polynomial in q = |k|^2 (Eq. (2): a derivative of order n becomes (ik)^n);
 *   - the semi-implicit step of Listing 1: the cubic term is evaluated pointwise in real space
 *     and transformed, the linear part is treated implicitly,
 *         S_k <- (S_k - dt q C_k) / (1 + dt q (eps + L(q))),   C = FFT(psi^3),
 *     (the listing's Laplacian and linear multipliers are -q and -q (eps + L(q))), followed by
 *     the inverse transform back to real space;
 *   - the discrete adjoint (transpose of the Jacobian) of that step, used for gradients;
 *   - the hydrodynamic PFC step of the multiphysics section (Eq. (5), (6), Listing 2);
 *   - the complex-amplitude form of the PFC model named at the end of that section (equations and
 *     readings with its code below).
 *
 * Readings where the paper is silent (each is listed with its reason in the design notes):
 *   - fields are real, so the spectral state is the half spectrum [n0][n1][n2/2+1]; after every
 *     forward transform and every update the two self-conjugate planes kx = 0 and kx = n2/2 are
 *     projected onto Hermitian symmetry, X(k) <- (X(k) + conj X(-k))/2.  In exact arithmetic this
 *     changes nothing; without it a half-spectrum state drifts away from any real field;
 *   - the correlation operator is parameterised as L(q) = (1-q)^2 for the one-mode model and
 *     L(q) = (1-q)^2 ((Q1^2 - q)^2 + R1) for the two-mode model (the paper's FCC operator is
 *     Q1^2 = 4/3, R1 = 0); the paper's undercooling eps is called r here;
 *   - wavenumbers k_j = 2 pi m_j / (n_j dx_j) with m_j in {0..n/2, -n/2+1..-1}.
 *
 * Arrays are C-order, last index fastest (x).  Complex arrays are interleaved (re, im) doubles.
 * Parallelism: OpenMP over independent lines and points only.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* pi to double precision (PI is not part of strict ISO C). */
static const double PI = 3.14159265358979323846264338327950288;

#define OR_OK 0
#define OR_ERR_ARG 1
#define OR_ERR_MEM 2

typedef struct {
    int ndim;          /* 1, 2 or 3 */
    int64_t n[3];      /* sizes, slowest axis first; n[ndim-1] is x */
    double dx[3];      /* grid spacing per axis */
    int model;         /* 0: one-mode, 1: two-mode */
    double r;          /* undercooling (the paper's epsilon) */
    double dt;         /* time step */
    double q1sq;       /* Q1^2 of the two-mode operator */
    double R1;         /* R1 of the two-mode operator */
    int linear_only;   /* 1: drop the cubic term (N = 0) */
    int no_projection; /* 1: skip the Hermitian projection (demonstrates the drift) */
} or_params;

/* Every axis even (so that kx = n/2 is a self-conjugate plane of the half spectrum) and >= 2. */
static int check_dims(int ndim, const int64_t *n)
{
    if (ndim < 1 || ndim > 3) return 0;
    for (int a = 0; a < ndim; ++a)
        if (n[a] < 2 || n[a] % 2 != 0) return 0;
    return 1;
}

static int64_t total_size(int ndim, const int64_t *n)
{
    int64_t t = 1;
    for (int a = 0; a < ndim; ++a) t *= n[a];
    return t;
}

/* ---------------------------------------------------------------- 1D FFT (recursive Cooley-Tukey) */

/* w[j] = exp(sign * 2 pi i j / N), j < N.  Each entry from cos/sin of its own angle. */
static cplx *twiddles(int64_t N, int sign)
{
    cplx *w = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    if (!w) return NULL;
    for (int64_t j = 0; j < N; ++j) {
        double ang = 2.0 * PI * (double)j / (double)N;
        w[j] = cos(ang) + (double)sign * sin(ang) * I;
    }
    return w;
}

/* Smallest prime factor of n >= 2. */
static int64_t smallest_factor(int64_t n)
{
    for (int64_t f = 2; f * f <= n; ++f)
        if (n % f == 0) return f;
    return n;
}

/* Decimation in time: out[0..n) = DFT of in[0], in[stride], ..., in[(n-1) stride], for the
 * top-level length N whose powers w[] holds; W_n^x = w[(x * wstep) mod N] with wstep = N / n.
 * With p the smallest prime factor of n and q = n / p, the p interleaved subsequences
 * in[r], in[r + p], ... (r < p) have q-point DFTs Y_r, and
 *     X[k + q s] = sum_{r < p} W_p^{r s} (W_n^{r k} Y_r[k]),   k < q, s < p.
 * p = 2 is the radix-2 butterfly X[k] = Y_0[k] + W_n^k Y_1[k], X[k + q] = Y_0[k] - W_n^k Y_1[k]. */
static void fft_rec(const cplx *in, int64_t stride, cplx *out, int64_t n, const cplx *w, int64_t wstep, int64_t N)
{
    if (n == 1) {
        out[0] = in[0];
        return;
    }
    const int64_t p = smallest_factor(n), q = n / p;
    for (int64_t r = 0; r < p; ++r) fft_rec(in + r * stride, p * stride, out + r * q, q, w, p * wstep, N);
    if (p == 2) {
        for (int64_t k = 0; k < q; ++k) {
            cplx e = out[k];
            cplx t = w[k * wstep] * out[k + q];
            out[k] = e + t;
            out[k + q] = e - t;
        }
        return;
    }
    cplx *t = (cplx *)malloc(sizeof(cplx) * (size_t)p);
    if (!t) abort();
    const int64_t wp = N / p; /* W_p^x = w[x * wp] */
    for (int64_t k = 0; k < q; ++k) {
        for (int64_t r = 0; r < p; ++r) t[r] = w[(r * k * wstep) % N] * out[r * q + k];
        for (int64_t s2 = 0; s2 < p; ++s2) {
            cplx acc = 0;
            for (int64_t r = 0; r < p; ++r) acc += w[((r * s2) % p) * wp] * t[r];
            out[k + q * s2] = acc;
        }
    }
    free(t);
}

/* In-place complex FFT along one axis of an nd complex array. sign = -1 forward, +1 inverse
 * (unnormalised). */
static int fft_axis(cplx *data, int ndim, const int64_t *n, int axis, int sign)
{
    int64_t len = n[axis];
    int64_t inner = 1;
    for (int a = axis + 1; a < ndim; ++a) inner *= n[a];
    int64_t lines = total_size(ndim, n) / len;
    cplx *w = twiddles(len, sign);
    if (!w) return OR_ERR_MEM;
    int err = 0;
#pragma omp parallel
    {
        cplx *src = (cplx *)malloc(sizeof(cplx) * (size_t)len);
        cplx *dst = (cplx *)malloc(sizeof(cplx) * (size_t)len);
        if (!src || !dst) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(static)
            for (int64_t l = 0; l < lines; ++l) {
                int64_t outer = l / inner, in = l % inner;
                cplx *base = data + outer * len * inner + in;
                for (int64_t j = 0; j < len; ++j) src[j] = base[j * inner];
                fft_rec(src, 1, dst, len, w, 1, len);
                for (int64_t j = 0; j < len; ++j) base[j * inner] = dst[j];
            }
        }
        free(src);
        free(dst);
    }
    free(w);
    return err ? OR_ERR_MEM : OR_OK;
}

static int fft_all_axes(cplx *data, int ndim, const int64_t *n, int sign)
{
    for (int a = 0; a < ndim; ++a) {
        int e = fft_axis(data, ndim, n, a, sign);
        if (e) return e;
    }
    return OR_OK;
}

/* Full complex nd FFT, in place on interleaved doubles.  sign = -1 forward, +1 inverse (no 1/N). */
int or_fft_c2c(int ndim, const int64_t *n, double *data, int sign)
{
    if (!check_dims(ndim, n) || (sign != 1 && sign != -1)) return OR_ERR_ARG;
    return fft_all_axes((cplx *)data, ndim, n, sign);
}

/* ---------------------------------------------------------------- half spectrum helpers */

/* Half-spectrum shape: same as n except the last axis, which has n/2+1 entries. */
static void half_dims(int ndim, const int64_t *n, int64_t *h)
{
    for (int a = 0; a < ndim; ++a) h[a] = n[a];
    h[ndim - 1] = n[ndim - 1] / 2 + 1;
}

/* Split a flat index over dims d into per-axis indices (C order). */
static void unflatten(int64_t idx, int ndim, const int64_t *d, int64_t *m)
{
    for (int a = ndim - 1; a >= 0; --a) {
        m[a] = idx % d[a];
        idx /= d[a];
    }
}

static int64_t flatten(int ndim, const int64_t *d, const int64_t *m)
{
    int64_t idx = 0;
    for (int a = 0; a < ndim; ++a) idx = idx * d[a] + m[a];
    return idx;
}

/* Hermitian projection of the planes kx = 0 and kx = n/2 of a half spectrum:
 * X(k) <- (X(k) + conj X(-k)) / 2, where -k negates every index modulo its axis length. */
static void project_hermitian(cplx *half, int ndim, const int64_t *n)
{
    int64_t h[3];
    half_dims(ndim, n, h);
    int64_t plane = total_size(ndim, n) / n[ndim - 1]; /* points per kx plane */
    int64_t kxs[2] = {0, n[ndim - 1] / 2};
    for (int s = 0; s < 2; ++s) {
        int64_t kx = kxs[s];
        /* Pair each point with its mirror once: visit p and compute its partner. */
        for (int64_t p = 0; p < plane; ++p) {
            int64_t m[3] = {0, 0, 0}, mm[3] = {0, 0, 0};
            unflatten(p * h[ndim - 1] + kx, ndim, h, m);
            for (int a = 0; a < ndim - 1; ++a) mm[a] = (n[a] - m[a]) % n[a];
            mm[ndim - 1] = kx;
            int64_t i0 = flatten(ndim, h, m), i1 = flatten(ndim, h, mm);
            if (i1 < i0) continue;
            cplx a = half[i0], b = half[i1];
            cplx v = 0.5 * (a + conj(b));
            half[i0] = v;
            half[i1] = conj(v);
        }
    }
}

/* Real-to-complex: full complex FFT of the real field, keep kx = 0..n/2, project. */
static int rfftn_impl(int ndim, const int64_t *n, const double *real, cplx *half, int project)
{
    int64_t N = total_size(ndim, n);
    cplx *full = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    if (!full) return OR_ERR_MEM;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) full[i] = real[i];
    int e = fft_all_axes(full, ndim, n, -1);
    if (e) {
        free(full);
        return e;
    }
    int64_t nx = n[ndim - 1], hx = nx / 2 + 1;
    int64_t rows = N / nx;
#pragma omp parallel for schedule(static)
    for (int64_t row = 0; row < rows; ++row)
        for (int64_t kx = 0; kx < hx; ++kx) half[row * hx + kx] = full[row * nx + kx];
    free(full);
    if (project) project_hermitian(half, ndim, n);
    return OR_OK;
}

/* Complex-to-real: rebuild the full spectrum by X(k) = conj X(-k) for kx > n/2, inverse FFT,
 * keep the real part, scale by 1/N. */
static int irfftn_impl(int ndim, const int64_t *n, const cplx *half, double *real)
{
    int64_t N = total_size(ndim, n);
    int64_t h[3];
    half_dims(ndim, n, h);
    cplx *full = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    if (!full) return OR_ERR_MEM;
    int64_t nx = n[ndim - 1];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        int64_t m[3] = {0, 0, 0}, mm[3] = {0, 0, 0};
        unflatten(i, ndim, n, m);
        if (m[ndim - 1] <= nx / 2) {
            full[i] = half[flatten(ndim, h, m)];
        } else {
            for (int a = 0; a < ndim; ++a) mm[a] = (n[a] - m[a]) % n[a];
            full[i] = conj(half[flatten(ndim, h, mm)]);
        }
    }
    int e = fft_all_axes(full, ndim, n, +1);
    if (e) {
        free(full);
        return e;
    }
    double inv = 1.0 / (double)N;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) real[i] = creal(full[i]) * inv;
    free(full);
    return OR_OK;
}

int or_rfftn(int ndim, const int64_t *n, const double *real, double *half)
{
    if (!check_dims(ndim, n)) return OR_ERR_ARG;
    return rfftn_impl(ndim, n, real, (cplx *)half, 1);
}

int or_irfftn(int ndim, const int64_t *n, const double *half, double *real)
{
    if (!check_dims(ndim, n)) return OR_ERR_ARG;
    return irfftn_impl(ndim, n, (const cplx *)half, real);
}

/* ---------------------------------------------------------------- PFC operator */

static int check_params(const or_params *p)
{
    if (!p || !check_dims(p->ndim, p->n)) return 0;
    if (p->model != 0 && p->model != 1) return 0;
    for (int a = 0; a < p->ndim; ++a)
        if (!(p->dx[a] > 0)) return 0;
    return 1;
}

/* Wavenumber of index m on an axis of length n with spacing dx. */
static double wavenumber(int64_t m, int64_t n, double dx)
{
    int64_t s = (m <= n / 2) ? m : m - n;
    return 2.0 * PI * (double)s / ((double)n * dx);
}

/* q = |k|^2 at half-spectrum point idx. */
static double q_at(const or_params *p, int64_t idx)
{
    int64_t h[3], m[3] = {0, 0, 0};
    half_dims(p->ndim, p->n, h);
    unflatten(idx, p->ndim, h, m);
    double q = 0.0;
    for (int a = 0; a < p->ndim; ++a) {
        double k = wavenumber(m[a], p->n[a], p->dx[a]);
        q += k * k;
    }
    return q;
}

/* Correlation operator as a polynomial in q (Eq. (3) with the derivative rule of Eq. (2)). */
static double corr_op(const or_params *p, double q)
{
    double a = (1.0 - q) * (1.0 - q);
    if (p->model == 0) return a;
    double b = (p->q1sq - q) * (p->q1sq - q);
    return a * (b + p->R1);
}

static int64_t half_size(int ndim, const int64_t *n)
{
    return total_size(ndim, n) / n[ndim - 1] * (n[ndim - 1] / 2 + 1);
}

int or_state_init(const or_params *p, const double *psi0, double *state)
{
    if (!check_params(p)) return OR_ERR_ARG;
    return rfftn_impl(p->ndim, p->n, psi0, (cplx *)state, !p->no_projection);
}

/* nsteps semi-implicit steps (Listing 1).  psi: real field psi^n in, psi^{n+nsteps} out.
 * state: half spectrum S of psi^n, updated in place. */
int or_step(const or_params *p, double *psi, double *state, int64_t nsteps)
{
    if (!check_params(p) || nsteps < 0) return OR_ERR_ARG;
    int ndim = p->ndim;
    int64_t N = total_size(ndim, p->n), H = half_size(ndim, p->n);
    cplx *S = (cplx *)state;
    double *cube = (double *)malloc(sizeof(double) * (size_t)N);
    cplx *NF = (cplx *)malloc(sizeof(cplx) * (size_t)H);
    if (!cube || !NF) {
        free(cube);
        free(NF);
        return OR_ERR_MEM;
    }
    int e = OR_OK;
    for (int64_t s = 0; s < nsteps && !e; ++s) {
        /* nonlinear term, pointwise in real space, then transformed */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) cube[i] = p->linear_only ? 0.0 : psi[i] * psi[i] * psi[i];
        e = rfftn_impl(ndim, p->n, cube, NF, !p->no_projection);
        if (e) break;
        /* semi-implicit update (Eq. (4) in Fourier space: the Laplacian multiplies by -q, the linear
         * operator by -q (r + L(q)); the cube explicit, the linear part implicit):
         *     S <- (S - dt q C) / (1 + dt q (r + L(q))),   C = FFT(psi^3) */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < H; ++i) {
            double q = q_at(p, i);
            double den = 1.0 + p->dt * (q * (p->r + corr_op(p, q)));
            S[i] = (S[i] - (p->dt * q) * NF[i]) / den;
        }
        if (!p->no_projection) project_hermitian(S, ndim, p->n);
        e = irfftn_impl(ndim, p->n, S, psi);
    }
    free(cube);
    free(NF);
    return e;
}

/* Free energy, Eq. (3), on the grid (dV = prod dx):
 *   out[0] = F with the quadratic part from the spectrum: (1/(2N)) sum_k w_k (r + L(q_k)) |S_k|^2,
 *            w_k = 1 on the planes kx = 0 and kx = n/2, else 2 (the missing half of the spectrum);
 *   out[1] = F with the quadratic part in real space: sum_x psi/2 * [(r + L) psi](x), where the
 *            operator is applied spectrally to the transform of psi itself;
 *   out[2] = mean of psi from the k = 0 mode, S_0 / N.
 * The quartic part sum_x psi^4/4 is in both. */
int or_energy(const or_params *p, const double *psi, const double *state, double *out)
{
    if (!check_params(p) || !out) return OR_ERR_ARG;
    int ndim = p->ndim;
    int64_t N = total_size(ndim, p->n), H = half_size(ndim, p->n);
    int64_t nx = p->n[ndim - 1], hx = nx / 2 + 1;
    const cplx *S = (const cplx *)state;
    double dV = 1.0;
    for (int a = 0; a < ndim; ++a) dV *= p->dx[a];

    double quad = 0.0, quart = 0.0, quad_real = 0.0;
#pragma omp parallel for reduction(+ : quad) schedule(static)
    for (int64_t i = 0; i < H; ++i) {
        int64_t kx = i % hx;
        double w = (kx == 0 || kx == nx / 2) ? 1.0 : 2.0;
        double q = q_at(p, i);
        double a = creal(S[i]), b = cimag(S[i]);
        quad += w * (p->r + corr_op(p, q)) * (a * a + b * b);
    }
    quad /= 2.0 * (double)N;
#pragma omp parallel for reduction(+ : quart) schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double v = psi[i] * psi[i];
        quart += 0.25 * v * v;
    }
    cplx *P = (cplx *)malloc(sizeof(cplx) * (size_t)H);
    double *g = (double *)malloc(sizeof(double) * (size_t)N);
    if (!P || !g) {
        free(P);
        free(g);
        return OR_ERR_MEM;
    }
    int e = rfftn_impl(ndim, p->n, psi, P, 1);
    if (!e) {
        for (int64_t i = 0; i < H; ++i) P[i] *= (p->r + corr_op(p, q_at(p, i)));
        e = irfftn_impl(ndim, p->n, P, g);
    }
    if (!e) {
#pragma omp parallel for reduction(+ : quad_real) schedule(static)
        for (int64_t i = 0; i < N; ++i) quad_real += 0.5 * psi[i] * g[i];
    }
    free(P);
    free(g);
    if (e) return e;
    out[0] = dV * (quad + quart);
    out[1] = dV * (quad_real + quart);
    out[2] = creal(S[0]) / (double)N;
    return OR_OK;
}

/* Adjoint of one step.  The step, as a map of the real field, is
 *   psi^{n+1} = F^{-1}[ A .* (F psi^n - dt q .* F (psi^n)^3) ],   A = 1/(1 + dt q (r + L(q))),
 * whose Jacobian is S_A - dt S_A S_K diag(3 (psi^n)^2) with the real symmetric Fourier multipliers
 * S_A = F^{-1} A F and S_K = F^{-1} q F.  Its transpose applied to lam = lam^{n+1}:
 *   mu = S_A lam,  nu = S_K S_A lam,  lam^n = mu - 3 dt (psi^n)^2 .* nu.
 * The derivative of psi^{n+1} with respect to r is -dt S_K S_A psi^{n+1}, so the contribution of
 * this step to dL/dr is -dt <nu, psi^{n+1}>, added to *dLdr. */
int or_step_backward(const or_params *p, const double *psi_n, const double *psi_np1,
                     const double *lam_np1, double *lam_n, double *dLdr)
{
    if (!check_params(p)) return OR_ERR_ARG;
    int ndim = p->ndim;
    int64_t N = total_size(ndim, p->n), H = half_size(ndim, p->n);
    cplx *Lh = (cplx *)malloc(sizeof(cplx) * (size_t)H);
    cplx *Kh = (cplx *)malloc(sizeof(cplx) * (size_t)H);
    double *mu = (double *)malloc(sizeof(double) * (size_t)N);
    double *nu = (double *)malloc(sizeof(double) * (size_t)N);
    int e = OR_OK;
    if (!Lh || !Kh || !mu || !nu) e = OR_ERR_MEM;
    if (!e) e = rfftn_impl(ndim, p->n, lam_np1, Lh, !p->no_projection);
    if (!e) {
        for (int64_t i = 0; i < H; ++i) {
            double q = q_at(p, i);
            double A = 1.0 / (1.0 + p->dt * q * (p->r + corr_op(p, q)));
            Lh[i] *= A;
            Kh[i] = q * Lh[i];
        }
        e = irfftn_impl(ndim, p->n, Lh, mu);
    }
    if (!e) e = irfftn_impl(ndim, p->n, Kh, nu);
    if (!e) {
        double acc = 0.0;
        const double c = p->linear_only ? 0.0 : 3.0 * p->dt;
#pragma omp parallel for reduction(+ : acc) schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            lam_n[i] = mu[i] - c * psi_n[i] * psi_n[i] * nu[i];
            acc += nu[i] * psi_np1[i];
        }
        if (dLdr) *dLdr += -p->dt * acc;
    }
    free(Lh);
    free(Kh);
    free(mu);
    free(nu);
    return e;
}

/* ---------------------------------------------------------------- hydrodynamic PFC */

/* Hydrodynamic PFC (section "Multiple GPU usage for Multiphysics PFC", Eq. (5) with the local
 * average of Eq. (6), time stepping of Listing 2).  Density psi and velocity v = (v_1 .. v_d),
 *     d_t psi = lap(dF/dpsi) - v . grad psi,
 *     rho0 d_t v = Gamma lap v - < psi grad(dF/dpsi) >,
 * dF/dpsi = (r + L)psi + psi^3, <.> a Gaussian average of width a0, in Fourier space the factor
 * G(q) = exp(-a0^2 q / 2).  One step, density first (the velocity update then uses the new
 * density), with S the density's half spectrum, V_j that of v_j and A(q) = 1/(1 + dt q (r + L(q))):
 *     N = FFT(psi^3),  T = FFT(sum_j v_j IFFT(D_j S))              (advection, explicit)
 *     S   <- A(q) (S - dt q N - dt T)
 *     M   =  FFT(psi^3) + (r + L(q)) S                             (chemical potential, new psi)
 *     V_j <- (V_j - (dt/rho0) G(q) FFT(psi IFFT(D_j M))) / (1 + (dt/rho0) Gamma q)
 * with D_j = i k_j the spectral first derivative.  Readings: k_j is taken as 0 at the Nyquist
 * index of each axis (a first derivative of a real field has no real Nyquist component); both
 * updates use the same dt; every spectrum is projected like the PFC state. */
typedef struct {
    double rho0;  /* mass density */
    double gamma; /* viscosity Gamma */
    double a0;    /* width of the Gaussian average (lattice spacing) */
} or_hydro;

/* wavenumber of index m with the Nyquist index mapped to 0 (first derivatives) */
static double odd_wavenumber(int64_t m, int64_t n, double dx)
{
    if (2 * m == n) return 0.0;
    return wavenumber(m, n, dx);
}

/* odd wavenumber of axis a at half-spectrum point idx */
static double kodd_at(const or_params *p, int64_t idx, int a)
{
    int64_t h[3], m[3] = {0, 0, 0};
    half_dims(p->ndim, p->n, h);
    unflatten(idx, p->ndim, h, m);
    return odd_wavenumber(m[a], p->n[a], p->dx[a]);
}

/* psi: real field; psi_state: its half spectrum; v: ndim real fields (component j at v + j N);
 * v_state: ndim half spectra (component j at v_state + 2 j H doubles).  All updated in place. */
int or_hydro_step(const or_params *p, const or_hydro *hp, double *psi, double *psi_state, double *v,
                  double *v_state, int64_t nsteps)
{
    if (!check_params(p) || !hp || !(hp->rho0 > 0.0) || nsteps < 0) return OR_ERR_ARG;
    const int ndim = p->ndim;
    const int64_t N = total_size(ndim, p->n), H = half_size(ndim, p->n);
    cplx *S = (cplx *)psi_state, *V = (cplx *)v_state;
    double *cube = (double *)malloc(sizeof(double) * (size_t)N), *a = (double *)malloc(sizeof(double) * (size_t)N),
           *tr = (double *)malloc(sizeof(double) * (size_t)N);
    cplx *NF = (cplx *)malloc(sizeof(cplx) * (size_t)H), *th = (cplx *)malloc(sizeof(cplx) * (size_t)H),
         *mu = (cplx *)malloc(sizeof(cplx) * (size_t)H);
    int e = (cube && a && tr && NF && th && mu) ? OR_OK : OR_ERR_MEM;
    const double dt = p->dt, c = p->dt / hp->rho0;
    for (int64_t st = 0; st < nsteps && !e; ++st) {
        /* density: cubic term and advection term, both transformed from real space */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            cube[i] = p->linear_only ? 0.0 : psi[i] * psi[i] * psi[i];
            a[i] = 0.0;
        }
        e = rfftn_impl(ndim, p->n, cube, NF, 1);
        for (int j = 0; j < ndim && !e; ++j) {
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < H; ++i) th[i] = I * kodd_at(p, i, j) * S[i];
            e = irfftn_impl(ndim, p->n, th, tr);
            if (e) break;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < N; ++i) a[i] += v[j * N + i] * tr[i];
        }
        if (!e) e = rfftn_impl(ndim, p->n, a, th, 1);
        if (e) break;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < H; ++i) {
            double q = q_at(p, i);
            double den = 1.0 + dt * (q * (p->r + corr_op(p, q)));
            S[i] = (S[i] - dt * (q * NF[i] + th[i])) / den;
        }
        project_hermitian(S, ndim, p->n);
        e = irfftn_impl(ndim, p->n, S, psi);
        if (e) break;
        /* velocity: M = FFT(psi^3) + (r + L) S of the new psi */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) cube[i] = p->linear_only ? 0.0 : psi[i] * psi[i] * psi[i];
        e = rfftn_impl(ndim, p->n, cube, mu, 1);
        if (e) break;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < H; ++i) mu[i] += (p->r + corr_op(p, q_at(p, i))) * S[i];
        for (int j = 0; j < ndim && !e; ++j) {
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < H; ++i) th[i] = I * kodd_at(p, i, j) * mu[i];
            e = irfftn_impl(ndim, p->n, th, tr);
            if (e) break;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < N; ++i) tr[i] *= psi[i];
            e = rfftn_impl(ndim, p->n, tr, th, 1);
            if (e) break;
            cplx *Vj = V + j * H;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < H; ++i) {
                double q = q_at(p, i);
                double G = exp(-0.5 * hp->a0 * hp->a0 * q);
                Vj[i] = (Vj[i] - c * G * th[i]) / (1.0 + c * hp->gamma * q);
            }
            project_hermitian(Vj, ndim, p->n);
            e = irfftn_impl(ndim, p->n, Vj, v + j * N);
        }
    }
    free(cube);
    free(a);
    free(tr);
    free(NF);
    free(th);
    free(mu);
    return e;
}

/* ---------------------------------------------------------------- amplitude equations */

/* Complex-amplitude (coarse-grained) PFC, the extension named at the end of the multiphysics
 * section: the density is written as psi = sum_j eta_j e^{i k_j.r} + c.c. over N principal
 * reciprocal-lattice vectors k_j, with slowly varying complex amplitudes eta_j.  The paper names
 * the formulation and leaves its equations to the cited overview of amplitude expansions; this
 * oracle takes the standard form of that literature with the free energy of Eq. (3) generalised by
 * the usual quadratic coefficient t:
 *     f(psi) = psi (dB + Bx (1 + lap)^2) psi / 2 - t psi^3 / 3 + v psi^4 / 4
 * (Eq. (3) is dB = r, Bx = 1, t = 0, v = 1), and for each amplitude
 *     d_t eta_j = -|k_j|^2 [ (dB + Bx (1 - |k_j|^2 + G_j)^2) eta_j + N_j ],   G_j = lap + 2 i k_j . grad,
 * where (1 - |k_j|^2 + G_j) is what (1 + lap) becomes on eta_j e^{i k_j.r} (it is G_j when |k_j| = 1),
 * where N_j is the resonant part of the nonlinearity -t psi^2 + v psi^3 at wave vector k_j:
 *     N_j = -t sum_{k_a + k_b = k_j} eta_a eta_b + v sum_{k_a + k_b + k_c = k_j} eta_a eta_b eta_c,
 * the sums running over ordered tuples of a, b, c in {+-1 .. +-N} with k_{-a} = -k_a and
 * eta_{-a} = conj(eta_a).  In Fourier space 1 - |k_j|^2 + G_j = 1 - |q + k_j|^2, and the
 * semi-implicit step (the update of Listing 1 applied to each amplitude) is
 *     eta_hat_j <- (eta_hat_j - dt |k_j|^2 FFT(N_j)) / (1 + dt |k_j|^2 (dB + Bx (1 - |q + k_j|^2)^2)),
 * followed by eta_j = IFFT(eta_hat_j).  Readings: the mean density is absorbed into dB, t, v; the
 * mobility is the long-wave -|k_j|^2; wave vectors q use numpy's fftfreq order (the Nyquist index
 * counts as -n/2, since G_j is odd in q); a tuple is resonant when its vector sum matches k_j to
 * 1e-9 times the largest |k_j|. */
#define OR_APFC_MAX 32
typedef struct {
    int ndim;
    int64_t n[3];
    double dx[3];
    int nfields;                  /* N <= 32 */
    double kvec[OR_APFC_MAX][3];  /* k_j, components along the grid axes (slowest first) */
    double dB, Bx, t, v, dt;
} or_apfc;

typedef struct {
    int nq, nc;   /* resonant ordered tuples for one field */
    int *q, *c;   /* signed field indices (+-(a+1)), 2 or 3 per tuple */
} apfc_terms;

static int apfc_check(const or_apfc *p)
{
    if (!p || !check_dims(p->ndim, p->n) || p->nfields < 1 || p->nfields > OR_APFC_MAX) return 0;
    for (int j = 0; j < p->nfields; ++j) {
        double kk = 0.0;
        for (int a = 0; a < p->ndim; ++a) kk += p->kvec[j][a] * p->kvec[j][a];
        if (!(kk > 0.0)) return 0;
    }
    return 1;
}

/* component a of k_s for a signed index s = +-(j+1) */
static double apfc_k(const or_apfc *p, int s, int a) { return s > 0 ? p->kvec[s - 1][a] : -p->kvec[-s - 1][a]; }

static int apfc_match(const or_apfc *p, const int *s, int len, int j, double tol)
{
    for (int a = 0; a < p->ndim; ++a) {
        double sum = 0.0;
        for (int i = 0; i < len; ++i) sum += apfc_k(p, s[i], a);
        if (fabs(sum - p->kvec[j][a]) > tol) return 0;
    }
    return 1;
}

/* All resonant ordered pairs and triples of every field (terms[j]). */
static int apfc_enumerate(const or_apfc *p, apfc_terms *terms)
{
    const int N = p->nfields, S = 2 * N;
    double kmax = 0.0;
    for (int j = 0; j < N; ++j) {
        double kk = 0.0;
        for (int a = 0; a < p->ndim; ++a) kk += p->kvec[j][a] * p->kvec[j][a];
        if (sqrt(kk) > kmax) kmax = sqrt(kk);
    }
    const double tol = 1e-9 * kmax;
    int sig[2 * OR_APFC_MAX];
    for (int i = 0; i < N; ++i) {
        sig[2 * i] = i + 1;
        sig[2 * i + 1] = -(i + 1);
    }
    for (int j = 0; j < N; ++j) {
        apfc_terms *T = &terms[j];
        T->nq = T->nc = 0;
        T->q = (int *)malloc(sizeof(int) * 2 * (size_t)S * S);
        T->c = (int *)malloc(sizeof(int) * 3 * (size_t)S * S * S);
        if (!T->q || !T->c) return OR_ERR_MEM;
        for (int x = 0; x < S; ++x)
            for (int y = 0; y < S; ++y) {
                int s[2] = {sig[x], sig[y]};
                if (apfc_match(p, s, 2, j, tol)) {
                    T->q[2 * T->nq] = s[0];
                    T->q[2 * T->nq + 1] = s[1];
                    ++T->nq;
                }
                for (int z = 0; z < S; ++z) {
                    int s3[3] = {sig[x], sig[y], sig[z]};
                    if (apfc_match(p, s3, 3, j, tol)) {
                        for (int i = 0; i < 3; ++i) T->c[3 * T->nc + i] = s3[i];
                        ++T->nc;
                    }
                }
            }
    }
    return OR_OK;
}

static void apfc_free(apfc_terms *terms, int N)
{
    for (int j = 0; j < N; ++j) {
        free(terms[j].q);
        free(terms[j].c);
    }
}

/* eta_s at point i of fields stored [N][P] */
static cplx apfc_eta(const cplx *eta, int64_t P, int64_t i, int s)
{
    return s > 0 ? eta[(int64_t)(s - 1) * P + i] : conj(eta[(int64_t)(-s - 1) * P + i]);
}

static void apfc_nonlinear_terms(const or_apfc *p, const apfc_terms *terms, const cplx *eta, cplx *out)
{
    const int64_t P = total_size(p->ndim, p->n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < P; ++i)
        for (int j = 0; j < p->nfields; ++j) {
            const apfc_terms *T = &terms[j];
            cplx sq = 0.0, sc = 0.0;
            for (int m = 0; m < T->nq; ++m) sq += apfc_eta(eta, P, i, T->q[2 * m]) * apfc_eta(eta, P, i, T->q[2 * m + 1]);
            for (int m = 0; m < T->nc; ++m)
                sc += apfc_eta(eta, P, i, T->c[3 * m]) * apfc_eta(eta, P, i, T->c[3 * m + 1]) *
                      apfc_eta(eta, P, i, T->c[3 * m + 2]);
            out[(int64_t)j * P + i] = -p->t * sq + p->v * sc;
        }
}

/* Signed wavenumber of index m on an axis of length n (numpy fftfreq order: Nyquist negative). */
static double apfc_wavenumber(int64_t m, int64_t n, double dx)
{
    int64_t s = (2 * m < n) ? m : m - n;
    return 2.0 * PI * (double)s / ((double)n * dx);
}

/* N_j at every point of the fields eta [N][grid] (complex). */
int or_apfc_nonlinear(const or_apfc *p, const double *eta, double *out)
{
    if (!apfc_check(p)) return OR_ERR_ARG;
    apfc_terms terms[OR_APFC_MAX];
    memset(terms, 0, sizeof terms);
    int e = apfc_enumerate(p, terms);
    if (!e) apfc_nonlinear_terms(p, terms, (const cplx *)eta, (cplx *)out);
    apfc_free(terms, p->nfields);
    return e;
}

/* Number of resonant ordered pairs and triples of field j (counts[0], counts[1]). */
int or_apfc_counts(const or_apfc *p, int j, int *counts)
{
    if (!apfc_check(p) || j < 0 || j >= p->nfields) return OR_ERR_ARG;
    apfc_terms terms[OR_APFC_MAX];
    memset(terms, 0, sizeof terms);
    int e = apfc_enumerate(p, terms);
    if (!e) {
        counts[0] = terms[j].nq;
        counts[1] = terms[j].nc;
    }
    apfc_free(terms, p->nfields);
    return e;
}

/* eta_hat_j = FFT(eta_j) for every field. */
int or_apfc_state_init(const or_apfc *p, const double *eta, double *eta_hat)
{
    if (!apfc_check(p)) return OR_ERR_ARG;
    const int64_t P = total_size(p->ndim, p->n);
    memcpy(eta_hat, eta, sizeof(cplx) * (size_t)(P * p->nfields));
    for (int j = 0; j < p->nfields; ++j) {
        int e = fft_all_axes((cplx *)eta_hat + (int64_t)j * P, p->ndim, p->n, -1);
        if (e) return e;
    }
    return OR_OK;
}

/* nsteps semi-implicit amplitude steps; eta (real space) and eta_hat (spectra) in place. */
int or_apfc_step(const or_apfc *p, double *eta_d, double *eta_hat_d, int64_t nsteps)
{
    if (!apfc_check(p) || nsteps < 0) return OR_ERR_ARG;
    const int ndim = p->ndim, N = p->nfields;
    const int64_t P = total_size(ndim, p->n);
    cplx *eta = (cplx *)eta_d, *S = (cplx *)eta_hat_d;
    cplx *nl = (cplx *)malloc(sizeof(cplx) * (size_t)(P * N));
    apfc_terms terms[OR_APFC_MAX];
    memset(terms, 0, sizeof terms);
    int e = nl ? apfc_enumerate(p, terms) : OR_ERR_MEM;
    for (int64_t st = 0; st < nsteps && !e; ++st) {
        apfc_nonlinear_terms(p, terms, eta, nl);
        for (int j = 0; j < N && !e; ++j) e = fft_all_axes(nl + (int64_t)j * P, ndim, p->n, -1);
        if (e) break;
        for (int j = 0; j < N; ++j) {
            double kk = 0.0;
            for (int a = 0; a < ndim; ++a) kk += p->kvec[j][a] * p->kvec[j][a];
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < P; ++i) {
                int64_t m[3] = {0, 0, 0};
                unflatten(i, ndim, p->n, m);
                double q2 = 0.0, kq = 0.0;
                for (int a = 0; a < ndim; ++a) {
                    double qa = apfc_wavenumber(m[a], p->n[a], p->dx[a]);
                    q2 += qa * qa;
                    kq += p->kvec[j][a] * qa;
                }
                double G = 1.0 - kk - q2 - 2.0 * kq; /* 1 - |q + k_j|^2 */
                int64_t o = (int64_t)j * P + i;
                S[o] = (S[o] - p->dt * kk * nl[o]) / (1.0 + p->dt * kk * (p->dB + p->Bx * G * G));
            }
        }
        memcpy(eta, S, sizeof(cplx) * (size_t)(P * N));
        for (int j = 0; j < N && !e; ++j) e = fft_all_axes(eta + (int64_t)j * P, ndim, p->n, 1);
        const double inv = 1.0 / (double)P;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < P * N; ++i) eta[i] *= inv;
    }
    apfc_free(terms, N);
    free(nl);
    return e;
}

/* Number of OpenMP threads the oracle would use (reported with the CPU baseline). */
int or_num_threads(void)
{
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            t = omp_get_num_threads();
#endif
        }
    }
    return t;
}

/* Sets the number of OpenMP threads of later calls (the CPU baseline is also timed on one). */
int or_set_num_threads(int n)
{
    if (n < 1) return OR_ERR_ARG;
#ifdef _OPENMP
    omp_set_num_threads(n);
#endif
    return OR_OK;
}
