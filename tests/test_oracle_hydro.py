"""Pins of the oracle's hydrodynamic PFC step (multiphysics section: Eq. (5), the Gaussian average
of Eq. (6), the time stepping of Listing 2) against things other than itself: the pinned PFC step
when the velocity is frozen, closed forms of the viscous decay and of linear advection, a
brute-force real-space evaluation of the Gaussian average of Eq. (6), and the reduction of a 3D run
that is constant along one axis to the 2D run."""
import numpy as np

import oracle
import pfc_inputs as P

DX = np.pi / 4


def relerr(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(np.asarray(b).ravel())


def spectra(v):
    return np.stack([oracle.rfftn(x) for x in v])


def kgrid(shape, dx=DX, odd=False):
    """Per-axis wavenumbers on the half spectrum from numpy's frequency grid; odd=True sets the
    Nyquist index to 0 (first derivatives of real fields)."""
    ks = []
    for a, n in enumerate(shape):
        k = 2 * np.pi * (np.fft.rfftfreq(n, d=dx) if a == len(shape) - 1 else np.fft.fftfreq(n, d=dx))
        if odd:
            k = k.copy()
            k[n // 2] = 0.0  # fftfreq puts -n/2 there, rfftfreq +n/2; either way it is the Nyquist index
        ks.append(k)
    return np.meshgrid(*ks, indexing="ij")


def test_frozen_velocity_reduces_to_the_pfc_step():
    """rho0 -> infinity freezes v at 0: the density then follows Listing 1 exactly."""
    shape = (16, 32)
    p = oracle.Params(shape, r=-0.25, dt=0.5)
    psi0 = P.pfc_initial_field(61, shape, -0.25)
    S0 = oracle.rfftn(psi0)
    v0 = np.zeros((2,) + shape)
    psi, S, v, V = oracle.hydro_step(p, oracle.Hydro(rho0=1e300, gamma=1.0, a0=1.0), psi0, S0, v0, spectra(v0), 12)
    ref_psi, ref_S = oracle.step(p, psi0, S0, 12)
    assert relerr(psi, ref_psi) < 1e-13 and relerr(S, ref_S) < 1e-13
    assert np.abs(v).max() < 1e-250


def test_uniform_density_viscous_decay_closed_form():
    """psi uniform: grad(dF/dpsi) = 0 and v . grad psi = 0, so psi stays put and every velocity mode
    decays by 1/(1 + dt Gamma q / rho0) per step."""
    shape = (8, 4, 16)
    p = oracle.Params(shape, r=-0.3, dt=0.5)
    psi0 = np.full(shape, -0.3)
    v0 = np.stack([P.uniform(62 + j, shape, -0.2, 0.2) for j in range(3)])
    V0 = spectra(v0)
    h = oracle.Hydro(rho0=2.0, gamma=0.7, a0=1.3)
    psi, S, v, V = oracle.hydro_step(p, h, psi0, oracle.rfftn(psi0), v0, V0, 5)
    q = sum(k * k for k in kgrid(shape))
    decay = (1.0 / (1.0 + 0.5 * 0.7 * q / 2.0)) ** 5
    assert np.abs(psi - psi0).max() < 1e-14
    assert relerr(V, V0 * decay[None]) < 1e-13


def test_linear_advection_closed_form():
    """Cubic term off, uniform frozen velocity c: each density mode is multiplied per step by
    (1 - dt i k.c) / (1 + dt q (r + L(q))), with k the first-derivative wavenumbers."""
    shape = (16, 32)
    c = (0.3, -0.45)
    p = oracle.Params(shape, r=-0.25, dt=0.5, linear_only=True)
    psi0 = P.pfc_initial_field(64, shape, -0.25)
    S0 = oracle.rfftn(psi0)
    v0 = np.stack([np.full(shape, c[0]), np.full(shape, c[1])])
    psi, S, v, V = oracle.hydro_step(p, oracle.Hydro(rho0=1e300, gamma=1.0, a0=1.0), psi0, S0, v0, spectra(v0), 6)
    ky, kx = kgrid(shape, odd=True)
    q = sum(k * k for k in kgrid(shape))
    factor = (1 - 0.5j * (ky * c[0] + kx * c[1])) / (1 + 0.5 * q * (-0.25 + (1 - q) ** 2))
    assert relerr(S, S0 * factor**6) < 1e-13
    assert relerr(psi, np.fft.irfftn(S0 * factor**6, shape, axes=(0, 1))) < 1e-13


def test_velocity_forcing_against_brute_force_gaussian_average():
    """One step from v = 0: the density step is the PFC step (v = 0 does not advect), then
    rho0 (v^1 - 0)/dt = Gamma lap v^1 - <psi^1 grad mu^1>.  The force psi grad mu is formed with numpy
    FFT derivatives, its Gaussian average of Eq. (6) is summed directly in real space over the
    periodic images, and the implicit viscous solve is applied with numpy's FFT."""
    shape = (8, 16)
    dt, rho0, gamma, a0, r = 0.5, 1.5, 0.8, 2.0 * DX, -0.25
    p = oracle.Params(shape, r=r, dt=dt)
    psi0 = P.pfc_initial_field(65, shape, r)
    v0 = np.zeros((2,) + shape)
    psi, S, v, V = oracle.hydro_step(p, oracle.Hydro(rho0=rho0, gamma=gamma, a0=a0), psi0, oracle.rfftn(psi0),
                                     v0, spectra(v0), 1)
    psi1, _ = oracle.step(p, psi0, oracle.rfftn(psi0), 1)
    # mu = dF/dpsi of psi^1 and its gradient, by numpy's FFT (derivative wavenumbers: Nyquist 0)
    q = sum(k * k for k in kgrid(shape))
    mu_hat = np.fft.rfftn(psi1**3) + (r + (1 - q) ** 2) * np.fft.rfftn(psi1)
    kyo, kxo = kgrid(shape, odd=True)
    force = [psi1 * np.fft.irfftn(1j * k * mu_hat, shape, axes=(0, 1)) for k in (kyo, kxo)]
    # Gaussian average: sum over grid points and periodic images of the normalised kernel
    ny, nx = shape
    Ly, Lx = ny * DX, nx * DX
    y = np.arange(ny) * DX
    x = np.arange(nx) * DX
    dy = y[:, None] - y[None, :]
    dxx = x[:, None] - x[None, :]
    gy = sum(np.exp(-((dy + m * Ly) ** 2) / (2 * a0 * a0)) for m in range(-6, 7))
    gx = sum(np.exp(-((dxx + m * Lx) ** 2) / (2 * a0 * a0)) for m in range(-6, 7))
    norm = DX * DX / (2 * np.pi * a0 * a0)
    for j in range(2):
        avg = norm * gy @ force[j] @ gx.T
        expect = np.fft.irfftn(np.fft.rfftn(-dt / rho0 * avg) / (1 + dt / rho0 * gamma * q), shape, axes=(0, 1))
        # the image sum and the spectral factor agree to ~1e-10 relative (kernel tails, aliasing)
        assert np.abs(v[j] - expect).max() < 1e-8 * np.abs(expect).max()
        assert np.abs(expect).max() > 1e-5  # the check is not vacuous


def test_3d_constant_along_an_axis_equals_2d():
    """A 3D run whose fields do not depend on z (v_z = 0) is the 2D run on every z plane."""
    shape2, nz = (8, 16), 4
    p2 = oracle.Params(shape2, r=-0.25, dt=0.5)
    p3 = oracle.Params((nz,) + shape2, r=-0.25, dt=0.5)
    psi2 = P.pfc_initial_field(66, shape2, -0.25)
    v2 = np.stack([P.uniform(67, shape2, -0.1, 0.1), P.uniform(68, shape2, -0.1, 0.1)])
    h = oracle.Hydro(rho0=1.0, gamma=1.0, a0=1.0)
    a = oracle.hydro_step(p2, h, psi2, oracle.rfftn(psi2), v2, spectra(v2), 4)
    psi3 = np.broadcast_to(psi2, (nz,) + shape2).copy()
    v3 = np.stack([np.zeros((nz,) + shape2)] + [np.broadcast_to(c, (nz,) + shape2).copy() for c in v2])
    b = oracle.hydro_step(p3, h, psi3, oracle.rfftn(psi3), v3, spectra(v3), 4)
    for zi in range(nz):
        assert np.abs(b[0][zi] - a[0]).max() < 1e-13
        assert np.abs(b[2][1][zi] - a[2][0]).max() < 1e-13 and np.abs(b[2][2][zi] - a[2][1]).max() < 1e-13
    assert np.abs(b[2][0]).max() < 1e-14
