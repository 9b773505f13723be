"""Pins of the FP64 CPU oracle against what the mathematics fixes.

Each test checks the oracle against something other than itself: the definition of the DFT
evaluated by brute force, numpy's FFT, closed forms of the linear PDE and of the free energy, the
PDE itself in the limit dt -> 0, exact invariants (mass, translation, tiling, uniform states) and,
for the adjoint, central finite differences of the forward oracle.  The method is arxiv 2603.26818:
Fourier pseudo-spectral discretisation (Eq. (2)), PFC energy (Eq. (3)) and dynamics (Eq. (4)),
semi-implicit update of Listing 1.
"""
import numpy as np
import pytest

import oracle
import pfc_inputs as P

DX = np.pi / 4


def brute_dft(f):
    """X(k) = sum_x f(x) exp(-2 pi i sum_a k_a x_a / n_a), as one dense matrix product."""
    E = np.ones((1, 1), complex)
    for n in f.shape:
        k = np.arange(n)
        E = np.kron(E, np.exp(-2j * np.pi * np.outer(k, k) / n))
    return (E @ f.ravel().astype(complex)).reshape(f.shape)


def half(X):
    return X[..., : X.shape[-1] // 2 + 1]


def relerr(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(np.asarray(b).ravel())


SHAPES = [(16,), (8, 4), (4, 8), (8, 16, 4), (4, 4, 8), (2, 8, 16),
          # lengths with factors 3, 5, 7 (the paper's grids 750 = 2 3 5^3 and 1400 = 2^3 5^2 7)
          (6,), (10,), (14,), (30,), (6, 10), (12, 14), (2, 6, 10), (10, 4, 6), (42,), (70, 2)]


# ------------------------------------------------------------------------------------ FFT pins
@pytest.mark.parametrize("shape", SHAPES)
def test_rfftn_equals_brute_force_dft(shape):
    f = P.normal(11, shape)
    assert relerr(oracle.rfftn(f), half(brute_dft(f))) < 1e-13


@pytest.mark.parametrize("shape", SHAPES)
def test_c2c_both_signs_equal_brute_force(shape):
    z = P.normal(12, shape) + 1j * P.normal(13, shape)
    assert relerr(oracle.fft_c2c(z, -1), brute_dft(z)) < 1e-13
    # inverse kernel e^{+ikx}: conj(DFT(conj z))
    assert relerr(oracle.fft_c2c(z, +1), np.conj(brute_dft(np.conj(z)))) < 1e-13


@pytest.mark.parametrize("shape", [(64, 32), (16, 32, 64), (128, 128), (32, 16, 8), (30, 20, 14), (750, 12),
                                   (12, 1400), (6, 10, 750), (150, 210)])
def test_rfftn_equals_numpy(shape):
    f = P.normal(14, shape)
    assert relerr(oracle.rfftn(f), np.fft.rfftn(f)) < 1e-13
    h = np.fft.rfftn(f)
    assert relerr(oracle.irfftn(h, shape), np.fft.irfftn(h, shape, axes=range(len(shape)))) < 1e-13


def test_single_mode_is_exact():
    shape = (16, 8, 32)
    m = (3, 1, 5)
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    phase = sum(2 * np.pi * mi * g / n for mi, g, n in zip(m, grids, shape))
    X = oracle.rfftn(np.cos(phase))
    N = np.prod(shape)
    expect = np.zeros_like(X)
    expect[m] = N / 2  # the +m bin; -m lies in the discarded half (kx = 27 > 16)
    assert np.abs(X - expect).max() < 1e-14 * N


@pytest.mark.parametrize("shape", [(8, 16, 4), (32, 64), (64,), (30, 20, 14), (750,), (28, 10)])
def test_parseval_roundtrip_linearity(shape):
    f, g = P.normal(15, shape), P.normal(16, shape)
    F, G = oracle.rfftn(f), oracle.rfftn(g)
    nx = shape[-1]
    w = np.full(F.shape[-1], 2.0)
    w[0] = 1.0
    w[nx // 2] = 1.0
    N = np.prod(shape)
    lhs, rhs = np.sum(f * f), np.sum(w * np.abs(F) ** 2) / N
    assert abs(lhs - rhs) / lhs < 1e-14
    assert np.abs(oracle.irfftn(F, shape) - f).max() < 1e-14
    assert relerr(oracle.rfftn(2.5 * f - 0.75 * g), 2.5 * F - 0.75 * G) < 1e-14


def test_shift_theorem():
    shape = (8, 16, 32)
    s = (3, 5, 7)
    f = P.normal(17, shape)
    F = oracle.rfftn(f)
    Fs = oracle.rfftn(np.roll(f, s, axis=(0, 1, 2)))
    k = np.meshgrid(*[np.arange(n) for n in F.shape], indexing="ij")
    ph = np.exp(-2j * np.pi * sum(ki * si / n for ki, si, n in zip(k, s, shape)))
    assert relerr(Fs, F * ph) < 1e-14


def test_self_conjugate_planes_are_exactly_hermitian():
    shape = (8, 16, 32)
    F = oracle.rfftn(P.normal(18, shape))
    for kx in (0, shape[-1] // 2):
        pl = F[:, :, kx]
        mirror = np.conj(pl[(-np.arange(8)) % 8][:, (-np.arange(16)) % 16])
        assert np.array_equal(pl, mirror)


def test_irfftn_discards_anti_hermitian_content():
    shape = (8, 16)
    F = oracle.rfftn(P.normal(19, shape))
    G = F.copy()
    G[3, 0] += 0.5j  # breaks the symmetry of the kx = 0 plane
    G[(-3) % 8, 0] += 0.5j
    assert np.abs(oracle.irfftn(G, shape) - oracle.irfftn(F, shape)).max() < 1e-15


# ------------------------------------------------------------------------------------ PFC pins
def kgrid_q(shape, dx=DX):
    """|k|^2 on the half spectrum, k = 2 pi m / (n dx), built here from numpy's frequency grid."""
    ks = [2 * np.pi * np.fft.fftfreq(n, d=dx) for n in shape[:-1]]
    ks.append(2 * np.pi * np.fft.rfftfreq(shape[-1], d=dx))
    grids = np.meshgrid(*ks, indexing="ij")
    return sum(g * g for g in grids)


@pytest.mark.parametrize("model,shape", [(0, (16, 32)), (1, (16, 32)), (0, (30, 14)), (1, (6, 10, 14))])
def test_linear_decay_closed_form(model, shape):
    """With the cubic term off, Eq. (4) is d/dt psi_k = -q (r + L(q)) psi_k per Fourier mode; the
    implicit linear step multiplies mode k by 1/(1 + dt q (r + L(q))) per step."""
    p = oracle.Params(shape, model=model, r=-0.25, dt=0.5, q1sq=2.0, R1=0.05, linear_only=True)
    psi0 = P.pfc_initial_field(1, shape, -0.25)
    S0 = oracle.rfftn(psi0)
    q = kgrid_q(shape)
    corr = (1 - q) ** 2 if model == 0 else (1 - q) ** 2 * ((2.0 - q) ** 2 + 0.05)
    growth = 1.0 / (1.0 + 0.5 * q * (-0.25 + corr))
    psi, S = oracle.step(p, psi0, S0, 7)
    assert relerr(S, S0 * growth**7) < 1e-13
    assert relerr(psi, np.fft.irfftn(S0 * growth**7, shape, axes=tuple(range(len(shape))))) < 1e-13


def test_step_consistent_with_pde_as_dt_to_zero():
    """(psi^1 - psi^0)/dt -> RHS of Eq. (4) for psi = c + a cos(k x), whose cube has modes k, 2k,
    3k, so the RHS has the closed form below."""
    shape = (8, 32)
    c, a, m = -0.2, 0.3, 2
    k = 2 * np.pi * m / (shape[1] * DX)
    x = np.arange(shape[1]) * DX
    X = np.broadcast_to(x, shape)
    psi0 = c + a * np.cos(k * X)
    r = -0.25
    q = k * k
    lin = -q * (r + (1 - q) ** 2) * a * np.cos(k * X)
    cub = (-(q) * (3 * c * c * a + 0.75 * a**3) * np.cos(k * X)
           - 4 * q * (1.5 * c * a * a) * np.cos(2 * k * X)
           - 9 * q * (0.25 * a**3) * np.cos(3 * k * X))
    rhs = lin + cub
    for dt in (1e-4, 1e-5):
        p = oracle.Params(shape, r=r, dt=dt)
        psi1, _ = oracle.step(p, psi0, oracle.rfftn(psi0), 1)
        est = (psi1 - psi0) / dt
        assert np.abs(est - rhs).max() < 50 * dt * np.abs(rhs).max()


def test_uniform_state_is_stationary_and_mass_bitwise():
    shape = (8, 16, 8)
    p = oracle.Params(shape, r=-0.3)
    psi0 = np.full(shape, -0.3)
    psi, S = oracle.step(p, psi0, oracle.rfftn(psi0), 10)
    assert np.abs(psi - psi0).max() < 1e-15
    psi0 = P.pfc_initial_field(2, shape, -0.3)
    S0 = oracle.state_init(p, psi0)
    psi, S = oracle.step(p, psi0, S0, 25)
    assert S[0, 0, 0] == S0[0, 0, 0]  # q = 0 at k = 0: the update leaves the mode untouched
    assert abs(psi.mean() - psi0.mean()) < 1e-15


def test_linearised_single_mode_growth():
    """Small mode eps*cos(kx) on a uniform background c: the cube contributes 3 c^2 eps cos(kx) to
    first order, so the one-step factor is (1 - 3 dt q c^2) / (1 + dt q (r + L(q))) + O(eps)."""
    shape = (4, 32)
    c, eps, m, r, dt = -0.25, 1e-7, 3, -0.25, 0.5
    k = 2 * np.pi * m / (shape[1] * DX)
    q = k * k
    psi0 = c + eps * np.cos(k * np.broadcast_to(np.arange(shape[1]) * DX, shape))
    p = oracle.Params(shape, r=r, dt=dt)
    _, S = oracle.step(p, psi0, oracle.rfftn(psi0), 1)
    S0 = oracle.rfftn(psi0)
    factor = (S[0, m] / S0[0, m]).real
    expect = (1 - 3 * dt * q * c * c) / (1 + dt * q * (r + (1 - q) ** 2))
    assert abs(factor - expect) < 1e-5 * abs(expect) + 1e-12


def test_translation_commutes_with_step():
    shape = (16, 8, 32)
    p = oracle.Params(shape, r=-0.3)
    psi0 = P.pfc_initial_field(3, shape, -0.3)
    a, _ = oracle.step(p, np.roll(psi0, (5, 3, 11), axis=(0, 1, 2)), oracle.rfftn(np.roll(psi0, (5, 3, 11), axis=(0, 1, 2))), 5)
    b, _ = oracle.step(p, psi0, oracle.rfftn(psi0), 5)
    assert np.abs(a - np.roll(b, (5, 3, 11), axis=(0, 1, 2))).max() < 1e-13


@pytest.mark.parametrize("small,reps", [((16, 16), (2, 4)), ((10, 6), (3, 5)), ((4, 6, 10), (7, 5, 3))])
def test_tiling_invariance(small, reps):
    """A field tiled k times along an axis evolves as the tiles of the small run (the big grid's
    spectrum lives on multiples of k); factors 3, 5, 7 exercise the non-radix-2 recursion."""
    big = tuple(n * k for n, k in zip(small, reps))
    p_small = oracle.Params(small, r=-0.25)
    p_big = oracle.Params(big, r=-0.25)
    psi0 = P.pfc_initial_field(4, small, -0.25)
    big0 = np.tile(psi0, reps)
    a, _ = oracle.step(p_small, psi0, oracle.rfftn(psi0), 20)
    b, _ = oracle.step(p_big, big0, oracle.rfftn(big0), 20)
    assert np.abs(np.tile(a, reps) - b).max() < 1e-13


# ------------------------------------------------------------------------------------ energy pins
def test_energy_closed_forms():
    shape = (16, 32)
    V = np.prod(shape) * DX * DX
    r = -0.3
    p = oracle.Params(shape, r=r)
    c = -0.3
    psi = np.full(shape, c)
    F, Freal, mean = oracle.energy(p, psi, oracle.rfftn(psi))
    expect = V * (0.5 * c * c * (r + 1.0) + 0.25 * c**4)  # L(0) = 1
    assert abs(F - expect) < 1e-13 * abs(expect) and abs(Freal - expect) < 1e-13 * abs(expect)
    assert abs(mean - c) < 1e-16
    a, m = 0.4, 5
    k = 2 * np.pi * m / (shape[1] * DX)
    psi = a * np.cos(k * np.broadcast_to(np.arange(shape[1]) * DX, shape))
    F, Freal, _ = oracle.energy(p, psi, oracle.rfftn(psi))
    # <cos^2> = 1/2, <cos^4> = 3/8
    expect = V * (0.25 * a * a * (r + (1 - k * k) ** 2) + 0.25 * 0.375 * a**4)
    assert abs(F - expect) < 1e-13 * abs(expect) and abs(Freal - expect) < 1e-13 * abs(expect)


def test_energy_forms_agree_and_decrease_128sq():
    """128^2 one-mode run (r = -0.25, dt = 0.5, psi0 = -0.25 + U(-0.1, 0.1), seed 1).  A sufficient
    condition for the semi-implicit step to decrease F is
        min_{q>0} [2/(dt q) + r + L(q)] >= 3 max|psi|^2  at both time levels;
    it is checked at every step, and F must not increase whenever it holds."""
    shape = (128, 128)
    p = oracle.Params(shape, r=-0.25, dt=0.5)
    psi = P.pfc_initial_field(1, shape, -0.25)
    S = oracle.state_init(p, psi)
    q = kgrid_q(shape)
    qpos = q[q > 0]
    bound = np.min(2.0 / (0.5 * qpos) - 0.25 + (1 - qpos) ** 2)
    F_prev, Freal, _ = oracle.energy(p, psi, S)
    assert abs(F_prev - Freal) < 1e-13 * abs(F_prev)
    checked = 0
    for n in range(100):
        m0 = np.abs(psi).max()
        psi, S = oracle.step(p, psi, S, 1)
        F, Freal, mean = oracle.energy(p, psi, S)
        assert abs(F - Freal) < 1e-12 * abs(F)
        if bound >= 3 * max(m0, np.abs(psi).max()) ** 2:
            assert F <= F_prev + 1e-12 * abs(F_prev)
            checked += 1
        F_prev = F
    assert checked == 100


def _anti_hermitian_kx0(S):
    """Norm of X(k) - conj X(-k) on the kx = 0 plane of a 2D half spectrum (0 for a real field)."""
    X0 = S[:, 0]
    mirror = np.conj(X0[(-np.arange(X0.shape[0])) % X0.shape[0]])
    return float(np.linalg.norm(X0 - mirror))


def test_half_spectrum_needs_the_hermitian_projection():
    """The projection of the self-conjugate planes (reading of the half-spectrum state; the paper
    keeps psi complex in MATLAB and never states one): the same 128^2 run as above, with and without
    it.  Without it, rounding-level anti-Hermitian content of the kx = 0 plane, which the inverse
    real transform discards, is multiplied by A(q) = 1/(1 + dt q (r + L(q))) > 1 at every step where
    r + L(q) < 0; it grows geometrically until the field itself blows up.  With it, that content is
    exactly zero, the run stays bounded and F does not increase."""
    shape = (128, 128)
    psi0 = P.pfc_initial_field(1, shape, -0.25)
    runs = {}
    for noproj in (True, False):
        p = oracle.Params(shape, r=-0.25, dt=0.5, no_projection=noproj)
        psi, S = psi0.copy(), oracle.state_init(p, psi0)
        hist = []
        for _ in range(24):  # 600 steps, recorded every 25
            psi, S = oracle.step(p, psi, S, 25)
            m = float(np.abs(psi).max())
            F, Freal, _ = oracle.energy(p, psi, S)
            hist.append((m, F, Freal, _anti_hermitian_kx0(S)))
            if not np.isfinite(m) or m > 10:
                break
        runs[noproj] = hist
    free, proj = runs[True], runs[False]
    # projected: exactly Hermitian, bounded, F non-increasing, both energy forms agree
    assert len(proj) == 24
    assert all(h[3] == 0.0 for h in proj)
    assert all(h[0] < 1.0 for h in proj)
    assert all(b[1] <= a[1] + 1e-12 * abs(a[1]) for a, b in zip(proj, proj[1:]))
    assert all(abs(h[1] - h[2]) < 1e-12 * abs(h[1]) for h in proj)
    # unprojected: anti-Hermitian content appears at rounding level and grows by many orders
    assert 0.0 < free[0][3] < 1e-10
    assert free[-1][3] > 1e6 * free[0][3] or not np.isfinite(free[-1][3])
    # ... while the field it steps still agrees with the projected run at first
    assert abs(free[0][0] - proj[0][0]) < 1e-12
    # it blows up within 600 steps: max|psi| > 10 or non-finite
    last = free[-1][0]
    assert not np.isfinite(last) or last > 10
    # and the spectral energy departs from the real-space one (the state no longer is a real
    # field's spectrum) before the field does
    assert any(np.isfinite(h[0]) and h[0] < 1.0 and abs(h[1] - h[2]) > 1e-3 * abs(h[2]) for h in free)


# ------------------------------------------------------------------------------------ adjoint pins
def _fd_jvp(p, psi, v, h=1e-2):
    """J v by central differences.  One step is a cubic polynomial map of psi, so the central
    difference is D(h) = J v + c h^2 exactly, and (4 D(h/2) - D(h)) / 3 = J v up to rounding."""
    S = lambda x: oracle.step(p, x, oracle.rfftn(x), 1)[0]
    D = lambda hh: (S(psi + hh * v) - S(psi - hh * v)) / (2 * hh)
    return (4 * D(h / 2) - D(h)) / 3


@pytest.mark.parametrize("shape", [(16, 16), (8, 4, 16)])
def test_adjoint_dot_product_against_fd(shape):
    p = oracle.Params(shape, r=-0.3, dt=0.5)
    psi = P.pfc_initial_field(5, shape, -0.3)
    psi1, _ = oracle.step(p, psi, oracle.rfftn(psi), 1)
    for t in range(3):
        v = P.normal(100 + t, shape)
        w = P.normal(200 + t, shape)
        jv = _fd_jvp(p, psi, v)
        jtw, _ = oracle.step_backward(p, psi, psi1, w)
        lhs, rhs = np.sum(jv * w), np.sum(v * jtw)
        assert abs(lhs - rhs) < 1e-11 * np.linalg.norm(jv) * np.linalg.norm(w)


def test_gradients_against_central_fd():
    shape = (16, 16)
    nsteps = 30
    p = oracle.Params(shape, r=-0.25, dt=0.5)
    psi0 = P.pfc_initial_field(5, shape, -0.25)
    target = oracle.rollout(oracle.Params(shape, r=-0.30, dt=0.5), psi0, nsteps)[-1]
    L, g, dLdr = oracle.loss_and_grad(p, psi0, target, nsteps)

    def loss(x, r):
        pp = oracle.Params(shape, r=r, dt=0.5)
        return float(np.sum((oracle.rollout(pp, x, nsteps)[-1] - target) ** 2))

    for t in range(4):
        v = P.normal(300 + t, shape)
        v /= np.linalg.norm(v)
        h = 1e-5
        fd = (loss(psi0 + h * v, -0.25) - loss(psi0 - h * v, -0.25)) / (2 * h)
        assert abs(fd - np.sum(g * v)) < 1e-6 * max(abs(fd), 1e-3 * np.linalg.norm(g))
    h = 1e-6
    fd_r = (loss(psi0, -0.25 + h) - loss(psi0, -0.25 - h)) / (2 * h)
    assert abs(fd_r - dLdr) < 1e-6 * abs(fd_r)
