"""pfc_step_noalloc (the step with the library's static device scratch) against pfc_step.

Both run the same kernels on the same inputs; only the location of the twiddle tables and of the
scratch spectrum differs, so the results must agree bit for bit.  Two calls in a row with different
plans (the second smaller, so the tables are re-uploaded and the spectrum area is partly reused),
then the first plan again, then a plan over the size limit (rejected, nothing launched)."""
import numpy as np
import pytest

from gpu_common import say, to_dev, to_np

pytestmark = pytest.mark.gpu


def _pair(shape, dtype, seed, r=-0.3):
    import paper_2603_26818_amd as pfc
    import pfc_inputs

    plan = pfc.Plan(shape, dtype=dtype, r=r, dt=0.5, device=0)
    psi0 = pfc_inputs.pfc_initial_field(seed, shape, r)
    psi_a = to_dev(psi0, dtype)
    st_a = plan.state_init(psi_a)
    psi_b = psi_a.clone()
    st_b = st_a.clone()
    return plan, (psi_a, st_a), (psi_b, st_b)


def _check_same(plan, a, b, nsteps, label):
    plan.step(a[0], a[1], nsteps)
    plan.step_noalloc(b[0], b[1], nsteps)
    pa, pb = to_np(a[0]), to_np(b[0])
    sa, sb = to_np(a[1]), to_np(b[1])
    assert np.all(np.isfinite(pb))
    nd = int(np.count_nonzero(pa != pb)) + int(np.count_nonzero(sa != sb))
    say(f"noalloc {label}: {nsteps} steps, differing values {nd}")
    assert nd == 0


def test_noalloc_matches_step_two_calls():
    say("noalloc: 3D (128, 64, 128) FP32, then 2D (64, 32) FP64, then the first plan again")
    plan1, a1, b1 = _pair((128, 64, 128), "f32", 31)
    _check_same(plan1, a1, b1, 4, "3D 128x64x128 FP32")
    plan2, a2, b2 = _pair((64, 32), "f64", 32, r=-0.25)
    _check_same(plan2, a2, b2, 3, "2D 64x32 FP64")
    # the first plan again: its tables are copied back in; continue both runs from where they are
    _check_same(plan1, a1, b1, 2, "3D 128x64x128 FP32, again")


def test_noalloc_largest_grid_and_limit():
    say("noalloc: 256^3 FP32 (the largest grid that fits), 2 steps")
    plan, a, b = _pair((256, 256, 256), "f32", 33)
    _check_same(plan, a, b, 2, "3D 256^3 FP32")
    import paper_2603_26818_amd as pfc

    big = pfc.Plan((256, 256, 256), dtype="f64", r=-0.3, dt=0.5, device=0)
    psi = big.empty_real().zero_()
    st = big.empty_state().zero_()
    with pytest.raises(pfc.PfcError) as ei:
        big.step_noalloc(psi, st, 1)
    assert ei.value.status == 4  # PFC_ERR_WORKSPACE
    say("noalloc: 256^3 FP64 rejected:", str(ei.value))
