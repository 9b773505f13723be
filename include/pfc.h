/*
 * pfc.h -- C ABI of the MI355X (gfx950) pseudo-spectral phase-field-crystal (PFC) library.
 *
 * The library advances the PFC equation of arxiv 2603.26818 (free energy Eq. (3), dynamics
 * Eq. (4)) with the Fourier pseudo-spectral method and the semi-implicit update of Listing 1:
 * each step transforms psi^3 to Fourier space (real-to-complex FFT), updates every mode with
 *     psi_hat <- (psi_hat - dt q FFT(psi^3)) / (1 + dt q (r + L(q))),   q = |k|^2,
 * and transforms back (complex-to-real FFT).  L(q) = (1-q)^2 (one-mode) or
 * (1-q)^2 ((Q1^2-q)^2 + R1) (two-mode; the paper's FCC operator is Q1^2 = 4/3, R1 = 0), r is the
 * paper's undercooling epsilon, and k_j = 2 pi m_j / (n_j dx_j) with m_j in {0..n/2, -n/2+1..-1}.
 *
 * Conventions shared by every entry point
 * - Arrays are C-order with x (the last index) fastest.  Real fields hold n0*n1*n2 (3D) or n0*n1
 *   (2D, x = n1) values of the plan's dtype.  Complex values are interleaved (re, im).
 * - "Natural" half spectra are [..][n_x/2+1] complex, unnormalised, forward sign e^{-ikx}.
 * - The spectral "state" carried between steps is in the library's own layout ("native"): the
 *   half spectrum with the self-conjugate planes kx = 0 and kx = n_x/2 folded into one complex
 *   plane, n_x/2 complex values per row.  3D grids pad rows longer than one 128-byte line to whole
 *   lines, and large power-of-two grids interleave blocks of 4 or 8 z planes line by line; the size
 *   is pfc_plan_state_bytes (the real field's bytes, plus any row padding).  Because any complex
 *   array in that layout corresponds to exactly one pair of Hermitian planes, the state always
 *   satisfies the symmetry of a real field.  Use pfc_state_export to read it.
 * - Device buffers and streams are owned by the caller; the plan owns only host metadata.  All
 *   device pointers must be 16-byte aligned and must not overlap unless an entry point says so.
 * - Every call is asynchronous on `stream` (a hipStream_t passed as void*, NULL = null stream) and
 *   runs on the plan's device.  Argument errors are returned synchronously and nothing is
 *   launched; kernel faults surface as PFC_ERR_HIP on a later call or synchronisation.
 * - No C++ exception crosses this interface.  pfc_last_error() gives a detail string for the
 *   calling thread's last failure.
 */
#ifndef PFC_H
#define PFC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PFC_OK = 0,
    PFC_ERR_INVALID_ARG = 1, /* bad value, NULL pointer, unstable dt, ...           */
    PFC_ERR_UNSUPPORTED = 2, /* unsupported grid size (see pfc_plan_create), ndim not 2/3 */
    PFC_ERR_ALIGNMENT = 3,   /* device pointer not 16-byte aligned                 */
    PFC_ERR_WORKSPACE = 4,   /* workspace missing or too small                     */
    PFC_ERR_HIP = 5,         /* a HIP runtime call failed                          */
    PFC_ERR_DIVERGED = 6,    /* non-finite energy or field detected                */
    PFC_ERR_INTERNAL = 7
} pfc_status;

typedef enum { PFC_F32 = 0, PFC_F64 = 1 } pfc_dtype;
typedef enum { PFC_ONE_MODE = 0, PFC_TWO_MODE = 1 } pfc_model;

/* flags */
#define PFC_FLAG_LINEAR_ONLY 1u /* drop the cubic term (FFT(psi^3) := 0): the linear PDE */
/* Layout hints of the native state (3D plans).  They change where values are stored, not the
 * arithmetic: every layout gives the same bits.  By default the library pairs z planes (blocks of
 * 2) on power-of-two grids with z >= 256 and planes of at least 1 MiB, where that measured faster.
 * PFC_FLAG_ZBLOCK(s) forces blocks of 2^s z planes, s in 0..3 (s > 0 needs rows of whole 128-byte
 * lines and a z length that is a power of two >= 256, or one whose last-axis schedules step by
 * multiples of 2^s, as 750's do for s = 1; else pfc_plan_create returns PFC_ERR_INVALID_ARG).
 * PFC_FLAG_XROWS_BLOCK makes the x passes visit the planes of a block in turn instead of the rows
 * in their natural order. */
#define PFC_FLAG_ZBLOCK(s) (0x10u | (((unsigned)(s) & 3u) << 5))
#define PFC_FLAG_XROWS_BLOCK 0x80u

typedef struct pfc_plan pfc_plan;

typedef struct {
    int ndim;        /* 2 or 3                                                    */
    int64_t n[3];    /* grid, slowest axis first; n[ndim-1] is x (sizes: below)   */
    double dx[3];    /* grid spacing per axis (> 0)                               */
    pfc_dtype dtype; /* arithmetic of fields, spectra and FFTs                    */
    pfc_model model; /* correlation operator L(q)                                 */
    double r;        /* undercooling (the paper's epsilon)                        */
    double dt;       /* time step (> 0)                                           */
    double q1sq;     /* Q1^2 of the two-mode operator (ignored for one-mode)      */
    double R1;       /* R1 of the two-mode operator (ignored for one-mode)        */
    int device;      /* HIP device ordinal the plan runs on                       */
    uint32_t flags;  /* PFC_FLAG_*                                                */
} pfc_plan_desc;

/* Validate `d` and create a plan (host memory only; no device allocation, no kernel).
 * Grid sizes: powers of two in [4, 2048]; or even sizes <= 2048 built from factors 2, 3, 5, 7 that
 * have a compiled schedule: for y and the last axis n in {6, 10, 12, 14, 20, 30, 60, 150, 700, 750,
 * 1400}, for x n/2 in {6, 10, 12, 14, 15, 20, 30, 60, 150, 375, 700, 750} (so the paper's 750^3 and
 * 1400^3 grids run).
 * Rejects: ndim not in {2,3}, any other size (UNSUPPORTED), dx <= 0,
 * dt <= 0, non-finite parameters, and any (r, dt) for which 1 + dt q (r + L(q)) <= 0 at some grid
 * wavevector (INVALID_ARG: the implicit denominator would vanish or change sign).
 * Source: the grid and wavenumbers of section "Fourier pseudo-spectral method" (Eq. (2)); the
 * operator of Eq. (3)-(4); the denominator of the update of Listing 1. */
pfc_status pfc_plan_create(pfc_plan **out, const pfc_plan_desc *d);

/* Bytes of device workspace the plan needs: one native spectrum (pfc_plan_state_bytes), the
 * twiddle table and the reduction partials.  The caller allocates it (>= 256-byte aligned).
 * Source: the transforms and spectral update of Listing 1 (their scratch). */
size_t pfc_plan_workspace_bytes(const pfc_plan *p);

/* Attach a caller-owned workspace and fill its twiddle table (host-computed in extended precision,
 * rounded once to the plan's dtype; one synchronous host-to-device copy).  Must be called before
 * any transform.  The workspace must stay valid, and unshared with concurrent calls, while the
 * plan uses it.  Source: the FFTs of Listing 1 (their twiddle factors). */
pfc_status pfc_plan_set_workspace(pfc_plan *p, void *dev_ptr, size_t bytes);

/* Change r and dt (re-validated as in pfc_plan_create).  Source: epsilon of Eq. (3)-(4) and the
 * time step of Listing 1. */
pfc_status pfc_plan_set_params(pfc_plan *p, double r, double dt);

/* Frees the plan's host memory (no device call).  Source: none in the paper (resource handling). */
pfc_status pfc_plan_destroy(pfc_plan *p);

/* Sizes in bytes of a real field, of a natural half spectrum and of a native state.  Source: the
 * real field psi and its Fourier coefficients of section "Fourier pseudo-spectral method". */
size_t pfc_plan_real_bytes(const pfc_plan *p);
size_t pfc_plan_half_bytes(const pfc_plan *p);
size_t pfc_plan_state_bytes(const pfc_plan *p);

/* Forward real-to-complex FFT of `real_in` into the natural half spectrum `half_out`
 * (unnormalised; the kx = 0 and kx = n_x/2 planes are exactly Hermitian).  Input preserved.
 * Source: the forward transform of section "Fourier pseudo-spectral method" and of Listing 1; the
 * paper states no sign or normalisation, MATLAB's are taken: e^{-ikx}, unnormalised. */
pfc_status pfc_fft_r2c(pfc_plan *p, const void *real_in, void *half_out, void *stream);

/* Inverse complex-to-real FFT of the natural half spectrum `half_in` into `real_out`, scaled by
 * 1/(total points).  The kx = 0 and kx = n_x/2 planes are first projected onto Hermitian symmetry,
 * X(k) <- (X(k) + conj X(-k))/2, so anti-Hermitian content is discarded.  Input preserved.
 * Source: the inverse transform of section "Fourier pseudo-spectral method" and of Listing 1
 * (MATLAB's convention: 1/N on the inverse). */
pfc_status pfc_fft_c2r(pfc_plan *p, const void *half_in, void *real_out, void *stream);

/* Spectral state of psi0 (its forward transform, native layout).  The k = 0 (mass) mode is
 * overwritten with an FP64 sum of psi0 rounded once to the dtype.  Source: Listing 1 starts from
 * psi and its transform; the paper keeps full complex spectra, so the half spectrum (whose
 * self-conjugate planes the packed layout keeps Hermitian) and the FP64 mass are this library's. */
pfc_status pfc_state_init(pfc_plan *p, const void *psi0, void *state, void *stream);

/* Copy the native state into a natural half spectrum [..][n_x/2+1].  Source: the Fourier
 * coefficients of section "Fourier pseudo-spectral method" (layout conversion only). */
pfc_status pfc_state_export(pfc_plan *p, const void *state, void *half_natural, void *stream);

/* Advance `nsteps` >= 0 semi-implicit steps (Listing 1).  psi: real field psi^n in, psi^{n+nsteps}
 * out.  state: native spectrum of psi^n in, updated in place.  The psi that enters a step is the
 * one the cube is taken of; the state is the one the update is applied to.  The intermediate
 * fields psi^{n+1} .. psi^{n+nsteps-1} are not stored where pfc_plan_x_fused says so (their
 * inverse and the next forward x transform then run as one pass); the results are the same bits.
 * Source: Eq. (4) stepped as in Listing 1 (cube, forward transform, semi-implicit update,
 * inverse transform). */
pfc_status pfc_step(pfc_plan *p, void *psi, void *state, int64_t nsteps, void *stream);

/* 1 when pfc_step fuses the inverse x transform of one step with the cube and forward x transform
 * of the next (x rows shorter than 1024 points whose default schedules fit a wavefront, on the
 * default x schedules), else 0 (also for p == NULL).  Its HBM traffic per step is then 10 field
 * passes, plus 2 per call, instead of 12 (3D; 2D: 6 plus 2 instead of 8).  Source: Listing 1
 * stores psi after every step; not storing it between the steps of one call is this library's. */
int pfc_plan_x_fused(const pfc_plan *p);

/* pfc_step for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same kernels and results as pfc_step, but
 * the twiddle tables and the scratch spectrum live in a static device array of the library
 * (65 MiB per GPU: 1 MiB of tables and a 64 MiB spectrum, allocated when the library's code is
 * loaded on that GPU and held until the process ends) instead of the plan's workspace, which need
 * not be attached.  Calls no hipMalloc or hipFree and allocates nothing.
 * Limit: the plan's native state must fit in 64 MiB (up to 256^3 FP32, or 2^23 points FP64);
 * larger plans get PFC_ERR_WORKSPACE and nothing is launched.  Arguments and errors otherwise as
 * pfc_step.  Every call on one GPU shares that GPU's array: calls that overlap in time on one GPU
 * (different streams without synchronisation, or threads) race and give wrong results.  The
 * plan's tables are copied into the array (an asynchronous copy on `stream` from host memory the
 * plan owns) when another plan used it last, so the plan must outlive its queued calls. */
pfc_status pfc_step_noalloc(pfc_plan *p, void *psi, void *state, int64_t nsteps, void *stream);

/* pfc_step with a divergence watchdog: after every `check_every` steps (and after the last) the FP64
 * energy and mean of (psi, state) are computed (as pfc_energy, into the workspace) and copied to the
 * host, which synchronises the stream.  A non-finite value stops the run with PFC_ERR_DIVERGED.
 * *done_steps receives the number of steps run.  Source: the step of Listing 1 and the energy of
 * Eq. (3). */
pfc_status pfc_step_watched(pfc_plan *p, void *psi, void *state, int64_t nsteps, int64_t check_every, void *stream,
                            int64_t *done_steps);

/* pfc_step with a HIP event recorded on `stream` around every kernel of every step, for
 * measurement.  pass_ms[i] receives the summed duration (ms) of pass i over all steps and *npasses
 * the number of passes per step: 3D 5 (x r2c with cube, y forward, z forward + update + z inverse,
 * y inverse, x c2r), 2D 3 (x r2c with cube, y forward + update + y inverse, x c2r).  pass_ms must
 * hold 5 doubles.  Synchronises the stream after each step; results equal those of pfc_step.
 * Source: the step of Listing 1 (timed). */
pfc_status pfc_step_timed(pfc_plan *p, void *psi, void *state, int64_t nsteps, void *stream, double *pass_ms,
                          int *npasses);

/* Autotuner: every pass of the step has a few candidate radix schedules compiled in (tile shapes
 * follow from the schedule: rows per workgroup of the x passes, column tiles of the strided passes).
 * Coordinate descent over whole steps: from the default schedules, each candidate of each pass in
 * turn is kept when `reps` runs of 4 steps (after one warm-up, events on `stream`) take less time,
 * so the choice accounts for the passes' interplay in a step, including the fused x pass between
 * steps (pfc_plan_x_fused), which needs the default x schedules.  The choice stays in the plan;
 * best_ms (5 doubles, may be NULL) receives the average time per pass of the choice, the passes run
 * apart as in pfc_step_timed.  psi_scratch (real field) and state_scratch (native state) are
 * caller-owned scratch of the plan's sizes: their contents are overwritten; they should hold a
 * finite field and its state (values do not change the timing).  Blocks until done.
 * Source: the transforms of Listing 1 (how they are scheduled; results do not depend on it beyond
 * rounding). */
pfc_status pfc_plan_autotune(pfc_plan *p, void *psi_scratch, void *state_scratch, void *stream, int reps,
                             double *best_ms);

/* The candidate chosen for each step pass (variants: 5 ints; *npasses as in pfc_step_timed), and
 * setting them back (e.g. from a cache of earlier tuning); set rejects out-of-range candidates.
 * Source: the transforms of Listing 1 (schedule choice). */
pfc_status pfc_plan_get_tuning(const pfc_plan *p, int *variants, int *npasses);
pfc_status pfc_plan_set_tuning(pfc_plan *p, const int *variants, int npasses);

/* Transpose of the Jacobian of one step, applied to lambda_np1 (the adjoint of psi^{n+1}):
 *     lambda_n = S_A lambda - 3 dt (psi_n)^2 .* S_K S_A lambda,
 * where S_A and S_K are the real symmetric Fourier multipliers A = 1/(1 + dt q (r + L(q))) and q.
 * Also adds this step's contribution to dL/dr, -dt <S_K S_A lambda, psi_np1>, to the FP64 device
 * scalar *dLdr_accum_dev.  lambda_n may be the same buffer as lambda_np1 (updated in place); it must
 * not overlap psi_n or psi_np1.  With PFC_FLAG_LINEAR_ONLY the cubic term is dropped.
 * Source: the update of Listing 1 (Eq. (4)), transposed; the paper has no adjoint.  In real space
 * one step is psi^{n+1} = S_A psi^n - dt S_A S_K (psi^n)^3, so its Jacobian's transpose is the
 * formula above (S_A and S_K are symmetric). */
pfc_status pfc_step_backward(pfc_plan *p, const void *psi_n, const void *psi_np1, const void *lambda_np1,
                             void *lambda_n, double *dLdr_accum_dev, void *stream);

/* Free energy, Eq. (3), on the grid: out_dev[0] = dV [ (1/(2N)) sum_k (r + L(q_k)) |psi_hat_k|^2
 * + sum_x psi^4/4 ] (sum over the full spectrum, dV = product of dx), out_dev[1] = mean of psi
 * from the k = 0 mode.  Accumulation in FP64 in both dtypes.  out_dev: 2 device doubles.
 * Source: Eq. (3) on the grid of section "Fourier pseudo-spectral method". */
pfc_status pfc_energy(pfc_plan *p, const void *psi, const void *state, double *out_dev, void *stream);

/* ---- Hydrodynamic PFC (section "Multiple GPU usage for Multiphysics PFC", Eq. (5), the Gaussian
 * average of Eq. (6), the time stepping of Listing 2) ----------------------------------------------
 * Density psi and velocity v = (v_0 .. v_{d-1}), component j along grid axis j (C order: axis 0 is
 * the slowest), d = ndim:
 *     d_t psi = lap(dF/dpsi) - v . grad psi,      rho0 d_t v = Gamma lap v - < psi grad(dF/dpsi) >,
 * dF/dpsi = (r + L)psi + psi^3 (the plan's model, r and dt), <.> the Gaussian average of width a0
 * (Fourier factor exp(-a0^2 q / 2)).  One step, psi first, then v from the new psi:
 *     psi_hat <- (psi_hat + dt (-q FFT(psi^3) - FFT(sum_j v_j IFFT(D_j psi_hat)))) / (1 + dt q (r + L))
 *     v_j_hat <- (v_j_hat - dt/rho0 G FFT(psi IFFT(D_j mu_hat))) / (1 + dt/rho0 Gamma q),
 *     mu_hat = FFT(psi^3) + (r + L) psi_hat,
 * D_j = i k_j the spectral first derivative with k_j = 0 at the Nyquist index. */
typedef struct {
    double rho0;  /* mass density, > 0 */
    double gamma; /* viscosity Gamma, >= 0 */
    double a0;    /* width of the Gaussian average (lattice spacing), >= 0 */
} pfc_hydro_params;

/* Device scratch the hydrodynamic step needs besides the plan's workspace: two native spectra and
 * two real fields (each 256-byte aligned).  Source: the transforms of Listing 2 (their scratch). */
size_t pfc_hydro_work_bytes(const pfc_plan *p);

/* States of psi and of the d velocity components (as pfc_state_init for each; Source: the spectra
 * Listing 2 starts from).  v: d real fields
 * back to back; v_state: d native states back to back (pfc_plan_real_bytes / _state_bytes apart). */
pfc_status pfc_hydro_state_init(pfc_plan *p, const void *psi, void *psi_state, const void *v, void *v_state,
                                void *stream);

/* Advance `nsteps` >= 0 hydrodynamic steps; psi, psi_state, v, v_state (layouts as above) are
 * updated in place.  work: caller-owned device scratch of at least pfc_hydro_work_bytes bytes,
 * 256-byte aligned, not overlapping the fields.  Returns PFC_ERR_INVALID_ARG for bad parameters,
 * PFC_ERR_WORKSPACE for a missing or short work buffer.  Source: Eq. (5)-(6) stepped as in
 * Listing 2. */
pfc_status pfc_hydro_step(pfc_plan *p, const pfc_hydro_params *hp, void *psi, void *psi_state, void *v,
                          void *v_state, void *work, size_t work_bytes, int64_t nsteps, void *stream);

/* ---- Batched form: many independent 2D runs of mixed sizes in one persistent launch ----------
 * Each instance is a 2D grid n0 x n1 (each a power of two in [32, 1024]) with its own model, r and
 * dt; all instances share the dtype and device.  pfc_batch_step advances every instance by nsteps
 * steps with ONE launch of a persistent kernel (replayed from a HIP graph captured on first use for
 * that nsteps): a step is three passes (x r2c with cube, y forward + update + y inverse, x c2r), each a
 * list of work items over all instances, separated by grid barriers.  The barrier wait is bounded:
 * if the workgroups cannot all be resident the launch ends early and pfc_batch_check reports it. */
typedef struct pfc_batch pfc_batch;

/* Validate `count` (1..256) 2D descriptors and create a batch (host memory only).  Source: each
 * instance is the step of Listing 1 (Eq. (4)) on its own grid.  Choices of the autotuner are not
 * cached here: the Python layer keeps them in a JSON file (Batch.autotune(cache_path=...)), so the
 * library does no file I/O. */
pfc_status pfc_batch_create(pfc_batch **out, const pfc_plan_desc *descs, int count);

/* Device workspace bytes: twiddle table, instance table, barrier state, one packed spectrum per
 * instance.  Source: the transforms of Listing 1, per instance (their scratch). */
size_t pfc_batch_workspace_bytes(const pfc_batch *b);

/* Bind the caller's fields: psi[i] (real, n0*n1) and state[i] (native spectrum, n0*n1/2 complex)
 * for instance i, and the workspace (>= 256-byte aligned).  Uploads the instance table and
 * twiddles and clears the barrier state (synchronous).  Drops graphs captured for earlier bindings.
 * Source: the fields psi and spectra of Listing 1, per instance. */
pfc_status pfc_batch_bind(pfc_batch *b, void *const *psi, void *const *state, void *workspace, size_t bytes);

/* state[i] = spectral state of psi[i] for every instance (as pfc_state_init).  Source: the
 * transform Listing 1 starts from, per instance. */
pfc_status pfc_batch_state_init(pfc_batch *b, void *stream);

/* Advance every instance by nsteps >= 0 steps: one graph launch of the persistent kernel.
 * Source: the step of Listing 1 (Eq. (4)), per instance. */
pfc_status pfc_batch_step(pfc_batch *b, int64_t nsteps, void *stream);

/* Synchronise `stream` and report whether a grid barrier of an earlier pfc_batch_step timed out
 * (PFC_ERR_INTERNAL; the barrier state is then cleared).  Source: none in the paper (error
 * reporting of the persistent launch). */
pfc_status pfc_batch_check(pfc_batch *b, void *stream);

/* Autotuner of the batched form: for each pass kind (x forward, y, x inverse) and each distinct
 * length among the instances, times every candidate radix schedule (which also sets the item shape:
 * rows per x item, pencils per y item) by launching the persistent kernel for `steps` steps, and
 * keeps the fastest.  THE BOUND FIELDS ARE ADVANCED by every trial: bind scratch fields to tune, then
 * copy the choice to the production batch with pfc_batch_get/set_tuning.  *ms_per_step (may be NULL)
 * receives the time per step of the final choice.  Blocks until done.  Source: the transforms of
 * Listing 1, per instance (schedule choice). */
pfc_status pfc_batch_autotune(pfc_batch *b, void *stream, int steps, double *ms_per_step);

/* Candidate per instance and pass: variants[3 i + k], k = 0 x forward, 1 y, 2 x inverse (caller's
 * instance order); n = 3 * count.  Setting re-uploads the instance table when bound.  Source: the
 * transforms of Listing 1 (schedule choice). */
pfc_status pfc_batch_get_tuning(const pfc_batch *b, int *variants, int n);
pfc_status pfc_batch_set_tuning(pfc_batch *b, const int *variants, int n);

/* Number of persistent workgroups of the batch launch (known after pfc_batch_bind).  Source: none
 * in the paper (launch shape). */
int pfc_batch_grid(const pfc_batch *b);

/* Frees the batch's host memory and its captured graphs.  Source: none in the paper (resource
 * handling). */
pfc_status pfc_batch_destroy(pfc_batch *b);

/* ---- Complex-amplitude form (the amplitude extension named at the end of the multiphysics
 * section; the paper gives no equations, so the standard amplitude expansion of the PFC energy is
 * taken) -------------------------------------------------------------------------------------------
 * The density is psi = sum_j eta_j e^{i k_j.r} + c.c. over N principal wave vectors k_j; the complex
 * amplitudes eta_j (N fields on one 2D or 3D periodic grid) follow
 *     d_t eta_j = -|k_j|^2 [ (dB + Bx (1 - |k_j|^2 + G_j)^2) eta_j + N_j ],   G_j = lap + 2 i k_j.grad,
 * where N_j is the resonant part of -t psi^2 + v psi^3 at k_j: the sum of -t eta_a eta_b over ordered
 * pairs with k_a + k_b = k_j and of v eta_a eta_b eta_c over ordered triples with k_a + k_b + k_c =
 * k_j, indices over +-1 .. +-N with k_{-a} = -k_a and eta_{-a} = conj(eta_a) (a vector sum matches
 * when it is within 1e-9 max|k| of k_j).  With dB = r, Bx = 1, t = 0, v = 1 this is the expansion of
 * the energy of Eq. (3).  One step (Listing 1's update applied to every amplitude):
 *     eta_hat_j <- (eta_hat_j - dt |k_j|^2 FFT(N_j)) / (1 + dt |k_j|^2 (dB + Bx (1 - |q + k_j|^2)^2)),
 *     eta_j = IFFT(eta_hat_j),
 * ((1 - |k_j|^2 + G_j) is (1 + lap) acting on eta_j e^{i k_j.r}; it is G_j on a unit shell), q on
 * numpy's fftfreq grid (the Nyquist index counts as -n/2: the operator is not even in q).
 * Layout: N complex grids back to back (field j at j * n0 n1 n2 elements), C order, interleaved
 * (re, im) in the plan's dtype; spectra in natural FFT order, same layout.  Unnormalised forward
 * transform, inverse with 1/(n0 n1 n2). */
#define PFC_APFC_MAX_FIELDS 32
typedef struct pfc_apfc pfc_apfc;
typedef struct {
    int ndim;                           /* 2 or 3 */
    int64_t n[3];                       /* grid, slowest axis first; each a power of two in [4, 2048]
                                           or one of 6, 10, 12, 14, 20, 30, 60, 150, 700, 750, 1400 */
    double dx[3];                       /* grid spacing per axis, > 0 */
    pfc_dtype dtype;
    int nfields;                        /* N, 1 .. PFC_APFC_MAX_FIELDS */
    double k[PFC_APFC_MAX_FIELDS][3];   /* k[j][a]: component of k_j along grid axis a (a < ndim) */
    double dB, Bx, t, v;                /* energy coefficients; Bx >= 0 */
    double dt;                          /* time step, > 0, with 1 + dt |k_j|^2 dB > 0 for every j */
    int device;                         /* HIP device of every pointer passed to this object */
} pfc_apfc_desc;

/* Validate the descriptor, find the resonant products of every amplitude (host memory only).
 * Source: the amplitude extension named at the end of section "Multiple GPU usage for
 * Multiphysics PFC" (the standard amplitude expansion of the energy of Eq. (3), written out
 * above). */
pfc_status pfc_apfc_create(pfc_apfc **out, const pfc_apfc_desc *d);

/* Bytes of the N fields (and of the N spectra): N n0 n1 n2 complex values.  Source: the
 * amplitudes of the amplitude extension named at the end of section "Multiple GPU usage for
 * Multiphysics PFC". */
size_t pfc_apfc_field_bytes(const pfc_apfc *p);

/* Device workspace bytes: twiddles, the product table, one scratch copy of the fields.  Source:
 * the transforms of Listing 1, applied to every amplitude (their scratch). */
size_t pfc_apfc_workspace_bytes(const pfc_apfc *p);

/* Attach a caller-owned device workspace (256-byte aligned); uploads the tables (synchronous).  The
 * workspace must stay valid while the object is used; calls on one object share its scratch, so
 * they must not run concurrently on different streams.  Source: the transforms of Listing 1,
 * applied to every amplitude (their twiddles). */
pfc_status pfc_apfc_set_workspace(pfc_apfc *p, void *dev_ptr, size_t bytes);

/* Number of distinct products that N_j sums one by one: pairs (t terms) and triples (v terms).
 * The triples that permute (j, i, -i), resonant on every lattice, are summed in closed form as
 * 3v (A^2 - |eta_j|^2) eta_j, A^2 = 2 sum_i |eta_i|^2, and are not counted; products whose
 * coefficient is zero are dropped.  Source: the resonant products of the amplitude expansion of
 * Eq. (3)'s energy (multiphysics section, amplitude extension). */
pfc_status pfc_apfc_terms(const pfc_apfc *p, int j, int *npairs, int *ntriples);

/* Complex FFT of every field over all axes, dir = -1 forward (unnormalised) or +1 inverse (times
 * 1/(n0 n1 n2)); in may equal out.  Source: the transforms of section "Fourier pseudo-spectral
 * method" on complex fields. */
pfc_status pfc_apfc_fft(pfc_apfc *p, const void *in, void *out, int dir, void *stream);

/* out_j = N_j at every point (out must not overlap eta).  Source: the resonant part of the
 * nonlinearity of Eq. (3)'s energy in the amplitude expansion (formula above). */
pfc_status pfc_apfc_nonlinear(pfc_apfc *p, const void *eta, void *out, void *stream);

/* eta_hat = forward FFT of eta (the state of the step).  Source: the transform Listing 1 starts
 * from, per amplitude. */
pfc_status pfc_apfc_state_init(pfc_apfc *p, const void *eta, void *eta_hat, void *stream);

/* Advance nsteps >= 0 steps; eta (real-space amplitudes) and eta_hat (their spectra) are updated
 * in place and must not overlap.  Source: the update of Listing 1 applied to every amplitude
 * (formula above). */
pfc_status pfc_apfc_step(pfc_apfc *p, void *eta, void *eta_hat, int64_t nsteps, void *stream);

/* Frees the object's host memory.  Source: none in the paper (resource handling). */
pfc_status pfc_apfc_destroy(pfc_apfc *p);

/* Name of a status code, and the calling thread's detail string of its last failure (valid until
 * the thread's next failing call).  Source: none in the paper (error reporting). */
const char *pfc_status_string(pfc_status st);
const char *pfc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PFC_H */
