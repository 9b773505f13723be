"""Parity on grids whose packed spectra use the blocked and padded layouts (Pack: rows padded to
whole 128-byte lines; blocks of 4 or 8 z planes interleaved by line on large power-of-two grids).
Every entry point that reads or writes the packed layout is compared with the FP64 oracle at a
size that selects it: the transforms (natural in and out), the state and its export, the step, the
energy, the adjoint step and the hydrodynamic step.  (The 2048^3 tiled-field test and the 512^3
benchmark-workload tests in test_gpu_fullsize.py run 8- and 4-plane blocks at full size.)"""
import numpy as np
import pytest

import oracle
import pfc_inputs as P
from gpu_common import TOL_FFT, TOL_STEP, fmt_errs, parity_errs, rounded, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pfc():
    import paper_2603_26818_amd as m

    m.load_library()
    return m


def _state_pitch(plan):
    return plan.state_shape[-1]


# (shape, dtype, layout flags): planes of 1 MiB (128 x 1024 FP32, 64 x 1024 FP64), so the default
# layout pairs z planes; then the hints: 4-plane blocks with the x passes in block order, 8-plane
# blocks
def _blocked():
    from paper_2603_26818_amd import _binding as B

    return [((256, 128, 2048), "f32", 0), ((256, 64, 2048), "f64", 0),
            ((256, 128, 2048), "f32", B.PFC_FLAG_ZBLOCK(2) | B.PFC_FLAG_XROWS_BLOCK),
            ((256, 64, 2048), "f64", B.PFC_FLAG_ZBLOCK(3)),
            # mixed radix: plane pairs of a 750-long z axis (its last-axis schedules, 15 10 5, step
            # by even element counts) with rows of 375 padded to whole lines
            ((750, 4, 750), "f32", B.PFC_FLAG_ZBLOCK(1)), ((750, 4, 750), "f64", B.PFC_FLAG_ZBLOCK(1))]


@pytest.mark.parametrize("case", range(6))
def test_blocked_layout_transforms_state_energy_step(pfc, case):
    shape, dtype, flags = _blocked()[case]
    say(f"[layout] {shape} {dtype} flags {flags:#x}: r2c, c2r, state, export, energy, 2 steps vs oracle")
    r = -0.30
    x = rounded(P.normal(41, shape), dtype)
    plan = pfc.Plan(shape, dtype=dtype, r=r, dt=0.5, flags=flags)
    X = plan.fft_r2c(to_dev(x, dtype))
    ref = oracle.rfftn(x)
    e_fwd = parity_errs(to_np(X), ref)
    y = to_np(plan.fft_c2r(X))
    e_inv = parity_errs(y, oracle.irfftn(ref, shape))
    del X
    say(f"      r2c {fmt_errs(e_fwd)}; c2r {fmt_errs(e_inv)}")
    assert max(e_fwd) < TOL_FFT[dtype] and max(e_inv) < TOL_FFT[dtype]
    psi0 = rounded(P.pfc_initial_field(42, shape, r), dtype)
    p = oracle.Params(shape, r=r, dt=0.5)
    S0 = oracle.state_init(p, psi0)
    psi = to_dev(psi0, dtype)
    st = plan.state_init(psi)
    e_st = parity_errs(to_np(plan.state_export(st)), S0)
    say(f"      state export {fmt_errs(e_st)}")
    assert max(e_st) < TOL_FFT[dtype]
    plan.step(psi, st, 2)
    ref_psi, ref_S = oracle.step(p, psi0, S0, 2)
    e = parity_errs(to_np(psi), ref_psi)
    es = parity_errs(to_np(plan.state_export(st)), ref_S)
    F = plan.energy(psi, st).cpu().tolist()
    Fr = oracle.energy(p, ref_psi, ref_S)
    say(f"      psi after 2 steps {fmt_errs(e)}; state {fmt_errs(es)}; energy {F[0]:.14g} vs {Fr[0]:.14g}")
    tol = TOL_STEP[dtype] if dtype == "f64" else 1e-5
    assert max(e) < tol and max(es) < tol
    # the energy is a sum over 2^25 modes (or points): its FP64 rounding shows in the difference of
    # the oracle's own two evaluations (spectral and real space, equal in exact arithmetic); the
    # GPU's sum, in another order, may differ from the oracle's by a few times that
    own = abs(Fr[0] - Fr[1]) / abs(Fr[0])
    tolF = max(tol, 10.0 * own)
    say(f"      energy rel diff {abs(F[0] - Fr[0]) / abs(Fr[0]):.2e} (oracle spectral vs real space {own:.2e})")
    assert abs(F[0] - Fr[0]) < tolF * abs(Fr[0]) and abs(F[1] - Fr[2]) < tol * abs(Fr[2])
    M, cb = shape[-1] // 2, (16 if dtype == "f32" else 8)  # columns of one 128-byte line
    assert _state_pitch(plan) == (M if M % cb == 0 else (M + cb - 1) // cb * cb)  # rows padded to whole lines


@pytest.mark.parametrize("hint", ["default", "zblock4_block_order"])
def test_blocked_layout_adjoint_and_hydro_fp64(pfc, hint):
    from paper_2603_26818_amd import _binding as B

    flags = 0 if hint == "default" else B.PFC_FLAG_ZBLOCK(2) | B.PFC_FLAG_XROWS_BLOCK
    shape, dtype, r = (256, 64, 2048), "f64", -0.30
    say(f"[layout] {shape} {dtype} flags {flags:#x}: adjoint step and hydrodynamic step vs oracle")
    p = oracle.Params(shape, r=r, dt=0.5)
    psi0 = P.pfc_initial_field(43, shape, r)
    psi1, _ = oracle.step(p, psi0, oracle.state_init(p, psi0), 1)
    lam = P.normal(44, shape)
    plan = pfc.Plan(shape, dtype=dtype, r=r, dt=0.5, flags=flags)
    got, dr = plan.step_backward(to_dev(psi0, dtype), to_dev(psi1, dtype), to_dev(lam, dtype))
    ref_lam, ref_dr = oracle.step_backward(p, psi0, psi1, lam)
    e = parity_errs(to_np(got), ref_lam)
    er = abs(float(dr[0].item()) - ref_dr) / abs(ref_dr)
    say(f"      adjoint step {fmt_errs(e)}; dL/dr rel {er:.2e}")
    assert max(e) < 1e-12 and er < 1e-12
    del got, plan
    hp = (1.0, 1.0, 1.0)
    ph = oracle.Params(shape, r=r, dt=0.25)
    v0 = np.stack([P.uniform(450 + j, shape, -0.05, 0.05) for j in range(3)])
    ref = oracle.hydro_step(ph, oracle.Hydro(*hp), psi0, oracle.rfftn(psi0), v0,
                            np.stack([oracle.rfftn(x) for x in v0]), 1)
    plan = pfc.Plan(shape, dtype=dtype, r=r, dt=0.25, flags=flags)
    psi, v = to_dev(psi0, dtype), to_dev(v0, dtype)
    S, V = plan.hydro_state_init(psi, v)
    plan.hydro_step(psi, S, v, V, 1, *hp)
    errs = [parity_errs(to_np(psi), ref[0])] + [parity_errs(to_np(v[j]), ref[2][j]) for j in range(3)]
    say("      hydro psi, v0, v1, v2: " + "; ".join(fmt_errs(x) for x in errs))
    assert max(max(x) for x in errs) < 1e-12


# mixed-radix rows longer than one line: M = 700 is padded to 704 (FP32 and FP64), M = 375 to 384
# (FP32) or 376 (FP64)
PADDED = [((12, 10, 1400), "f32"), ((12, 10, 1400), "f64"), ((10, 6, 750), "f32"), ((10, 6, 750), "f64")]


@pytest.mark.parametrize("shape,dtype", PADDED)
def test_padded_rows(pfc, shape, dtype):
    say(f"[layout] {shape} {dtype}: padded rows, 5 steps, r2c, export vs oracle")
    r = -0.30
    plan = pfc.Plan(shape, dtype=dtype, r=r, dt=0.5)
    M, cb = shape[-1] // 2, 16 if dtype == "f32" else 8
    assert _state_pitch(plan) == -(-M // cb) * cb
    x = rounded(P.normal(46, shape), dtype)
    e_fwd = parity_errs(to_np(plan.fft_r2c(to_dev(x, dtype))), oracle.rfftn(x))
    psi0 = rounded(P.pfc_initial_field(47, shape, r), dtype)
    p = oracle.Params(shape, r=r, dt=0.5)
    ref_psi, ref_S = oracle.step(p, psi0, oracle.state_init(p, psi0), 5)
    psi = to_dev(psi0, dtype)
    st = plan.state_init(psi)
    plan.step(psi, st, 5)
    e = parity_errs(to_np(psi), ref_psi)
    es = parity_errs(to_np(plan.state_export(st)), ref_S)
    # one adjoint step: its nu spectrum shares the output buffer, in rows of M (not the padded pitch)
    lam = rounded(P.normal(48, shape), dtype)
    got, dr = plan.step_backward(to_dev(psi0, dtype), to_dev(rounded(ref_psi, dtype), dtype), to_dev(lam, dtype))
    ref_lam, ref_dr = oracle.step_backward(p, psi0, rounded(ref_psi, dtype), lam)
    eb = parity_errs(to_np(got), ref_lam)
    er = abs(float(dr[0].item()) - ref_dr) / abs(ref_dr)
    say(f"      r2c {fmt_errs(e_fwd)}; psi {fmt_errs(e)}; state {fmt_errs(es)}; adjoint step {fmt_errs(eb)}, "
        f"dL/dr {er:.1e}")
    assert max(e_fwd) < TOL_FFT[dtype] and max(e) < TOL_STEP[dtype] and max(es) < TOL_STEP[dtype]
    tolb = 1e-12 if dtype == "f64" else 5e-6
    assert max(eb) < tolb and er < 10 * tolb  # dL/dr: a sum over all points, as test_gpu_step.py
