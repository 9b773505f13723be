"""Pins of the oracle's complex-amplitude PFC step (the amplitude form named at the end of the
multiphysics section; equations and readings in pfc_oracle.c) against things other than itself:
the textbook closed form of the triangular-lattice nonlinearity, a brute-force projection of
-t psi^2 + v psi^3 onto each principal mode over a periodic unit cell, the equilibrium amplitude
of a uniform crystal, the closed-form linear decay of every mode, the covariance of the step under
a rigid translation of the crystal, and the reduction of a z-independent 3D run to the 2D run."""
import numpy as np
import pytest

import oracle
import pfc_inputs as P


def relerr(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(np.asarray(b).ravel())


def random_amplitudes(seed, nfields, shape):
    return P.amplitude_fields(seed, nfields, shape, 0.0, 1.0)


@pytest.mark.parametrize("t", [0.0, 0.5])
def test_triangular_nonlinearity_closed_form(t):
    """One triangular shell: N_j = 3v (A^2 - |eta_j|^2) eta_j - 2t prod_{i != j} conj(eta_i),
    A^2 = 2 sum |eta_i|^2 (the standard form of the amplitude-expansion literature)."""
    a = oracle.Apfc((4, 6), P.lattice_vectors("triangular"), t=t, v=0.7)
    eta = random_amplitudes(71, 3, (4, 6))
    N = oracle.apfc_nonlinear(a, eta)
    A2 = 2 * np.sum(np.abs(eta) ** 2, axis=0)
    for j in range(3):
        others = [np.conj(eta[i]) for i in range(3) if i != j]
        ref = 3 * 0.7 * (A2 - np.abs(eta[j]) ** 2) * eta[j] - 2 * t * others[0] * others[1]
        assert np.abs(N[j] - ref).max() < 1e-13 * np.abs(ref).max()
    # resonance counts: ordered pairs (k_a + k_b = k_j) and ordered triples
    assert [oracle.apfc_counts(a, j) for j in range(3)] == [(2, 15)] * 3


def unit_cell(name):
    """A periodic box on which every e^{i k_j . r} of the lattice is periodic, sampled finely enough
    that a cubic polynomial in those exponentials is integrated exactly; returns (axes coordinates)."""
    k = P.lattice_vectors(name)
    s3 = np.sqrt(3.0) / 2
    if name in ("triangular", "triangular2"):
        box, n = (4 * np.pi, 2 * np.pi / s3), (24, 24)
    elif name.startswith("triangular"):  # up to |k| = 4: indices |2i - j| <= 8 along y, |j| <= 5 along x
        box, n = (4 * np.pi, 2 * np.pi / s3), (64, 32)
    elif name == "square":
        box, n = (2 * np.pi, 2 * np.pi), (8, 8)
    elif name == "bcc":
        box, n = (2 * np.pi * np.sqrt(2),) * 3, (8, 8, 8)
    else:  # fcc2: components are multiples of 1/sqrt(3)
        box, n = (2 * np.pi * np.sqrt(3),) * 3, (16, 16, 16)
    # every k . r must be periodic on the box
    for kj in k:
        for a in range(len(box)):
            m = kj[a] * box[a] / (2 * np.pi)
            assert abs(m - round(m)) < 1e-12
    axes = [np.arange(nn) * L / nn for nn, L in zip(n, box)]
    return np.meshgrid(*axes, indexing="ij")


@pytest.mark.parametrize("name", ["triangular", "square", "triangular2", "bcc", "fcc2", "triangular30"])
def test_nonlinearity_equals_projection_of_the_density_nonlinearity(name):
    """For constant amplitudes, N_j is the Fourier coefficient at k_j of -t psi^2 + v psi^3 with
    psi = sum_j eta_j e^{i k_j.r} + c.c.: computed here by sampling psi on a periodic cell of the
    lattice and averaging f(psi) e^{-i k_j.r} (exact for these trigonometric polynomials)."""
    k = P.lattice_vectors(name)
    nf, nd = k.shape
    t, v = 0.35, 0.8
    eta0 = random_amplitudes(72 + nf, nf, (1,))[:, 0]
    shape = (2,) * nd
    a = oracle.Apfc(shape, k, t=t, v=v)
    eta = np.broadcast_to(eta0.reshape((nf,) + (1,) * nd), (nf,) + shape).copy()
    N = oracle.apfc_nonlinear(a, eta)
    R = unit_cell(name)
    psi = np.zeros(R[0].shape)
    for j in range(nf):
        phase = sum(k[j, c] * R[c] for c in range(nd))
        psi += 2 * np.real(eta0[j] * np.exp(1j * phase))
    f = -t * psi**2 + v * psi**3
    for j in range(nf):
        phase = sum(k[j, c] * R[c] for c in range(nd))
        proj = np.mean(f * np.exp(-1j * phase))
        assert abs(N[j].ravel()[0] - proj) < 1e-12 * max(1.0, abs(proj)), (name, j)


def test_uniform_crystal_reaches_the_equilibrium_amplitude():
    """Uniform real amplitudes eta_j = phi on one triangular shell: G_j phi = 0, so
    phi <- (phi - dt (-2t phi^2 + 15 v phi^3)) / (1 + dt dB), whose stable fixed point is
    phi* = (t + sqrt(t^2 - 15 v dB)) / (15 v)."""
    dB, t, v = 0.02, 0.5, 1.0 / 3.0
    a = oracle.Apfc((4, 4), P.lattice_vectors("triangular"), dB=dB, t=t, v=v, dt=0.5)
    eta = np.full((3, 4, 4), 0.1, np.complex128)
    eta, S = oracle.apfc_step(a, eta, oracle.apfc_state_init(a, eta), 400)
    phi = (t + np.sqrt(t * t - 15 * v * dB)) / (15 * v)
    assert np.abs(eta - phi).max() < 1e-12
    # and one step from phi0 follows the scalar recursion exactly
    eta1, _ = oracle.apfc_step(a, np.full((3, 4, 4), 0.1 + 0j), oracle.apfc_state_init(a, np.full((3, 4, 4), 0.1 + 0j)), 1)
    ref = (0.1 - 0.5 * (-2 * t * 0.01 + 15 * v * 0.001)) / (1 + 0.5 * dB)
    assert np.abs(eta1 - ref).max() < 1e-15


def test_linear_modes_closed_form():
    """t = v = 0: every Fourier mode q of amplitude j is multiplied per step by
    1 / (1 + dt |k_j|^2 (dB + Bx (1 - |q + k_j|^2)^2)), with q on numpy's fftfreq grid (the one-mode
    operator (1 + lap)^2 acting on eta_j e^{i k_j.r}; two shells, so |k_j| = 1 and sqrt(3) occur)."""
    shape, dx = (8, 12), (np.pi / 2, np.pi / 3)
    k = P.lattice_vectors("triangular2")
    a = oracle.Apfc(shape, k, dx=dx, dB=-0.1, Bx=0.9, t=0.0, v=0.0, dt=0.4)
    eta0 = random_amplitudes(73, 6, shape)
    eta, S = oracle.apfc_step(a, eta0, oracle.apfc_state_init(a, eta0), 5)
    qy, qx = np.meshgrid(*[2 * np.pi * np.fft.fftfreq(n, d) for n, d in zip(shape, dx)], indexing="ij")
    for j in range(6):
        G = 1 - ((qy + k[j, 0]) ** 2 + (qx + k[j, 1]) ** 2)
        kk = k[j] @ k[j]
        ref = np.fft.fftn(eta0[j]) / (1 + 0.4 * kk * (-0.1 + 0.9 * G**2)) ** 5
        assert relerr(S[j], ref) < 1e-13
        assert relerr(eta[j], np.fft.ifftn(ref)) < 1e-13


@pytest.mark.parametrize("name,shape", [("triangular", (12, 8)), ("bcc", (4, 6, 8))])
def test_step_commutes_with_a_rigid_translation(name, shape):
    """Shifting the crystal by a uniform displacement u multiplies eta_j by exp(-i k_j.u); the
    free energy, hence the step, is covariant under it (this fixes every conjugation in N_j)."""
    k = P.lattice_vectors(name)
    nf, nd = k.shape
    a = oracle.Apfc(shape, k, dB=-0.2, t=0.4, v=0.9, dt=0.3)
    eta0 = P.amplitude_fields(74, nf, shape, 0.15, 0.05)
    u = np.array([0.7, -1.3, 2.1][:nd])
    ph = np.exp(-1j * (k @ u)).reshape((nf,) + (1,) * nd)
    e1, _ = oracle.apfc_step(a, eta0, oracle.apfc_state_init(a, eta0), 6)
    e2, _ = oracle.apfc_step(a, eta0 * ph, oracle.apfc_state_init(a, eta0 * ph), 6)
    assert relerr(e2, e1 * ph) < 1e-13
    # a phase pattern that is not a translation (when the lattice has resonant triads) breaks it
    if name == "triangular":
        bad = np.exp(1j * np.array([0.3, 0.0, 0.0])).reshape((nf,) + (1,) * nd)
        e3, _ = oracle.apfc_step(a, eta0 * bad, oracle.apfc_state_init(a, eta0 * bad), 6)
        assert relerr(e3, e1 * bad) > 1e-4


def test_3d_constant_along_an_axis_equals_2d():
    """Triangular amplitudes embedded in 3D (k_z = 0) with fields constant along z: every z plane
    follows the 2D run."""
    k2 = P.lattice_vectors("triangular")
    k3 = np.concatenate([np.zeros((3, 1)), k2], axis=1)
    a2 = oracle.Apfc((8, 12), k2, dB=-0.15, t=0.3, v=1.0, dt=0.5)
    a3 = oracle.Apfc((4, 8, 12), k3, dB=-0.15, t=0.3, v=1.0, dt=0.5)
    eta2 = P.amplitude_fields(75, 3, (8, 12), 0.1, 0.05)
    eta3 = np.broadcast_to(eta2[:, None], (3, 4, 8, 12)).copy()
    r2, _ = oracle.apfc_step(a2, eta2, oracle.apfc_state_init(a2, eta2), 5)
    r3, _ = oracle.apfc_step(a3, eta3, oracle.apfc_state_init(a3, eta3), 5)
    for z in range(4):
        assert np.abs(r3[:, z] - r2).max() < 1e-14
