"""Seeded input generator: counter form against the published sequential generator."""
import os

import numpy as np
import pytest

import pfc_inputs as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed1234567.txt")


def _golden():
    with open(GOLDEN) as f:
        return [int(l) for l in f if l.strip() and not l.startswith("#")]


def test_sequential_matches_reference_vector():
    assert P.splitmix64_sequential(1234567, 5) == _golden()


@pytest.mark.parametrize("seed", [0, 1, 1234567, 2**63 + 5, 2**64 - 1])
def test_counter_form_equals_sequential(seed):
    seq = P.splitmix64_sequential(seed, 300)
    ctr = P.splitmix64(seed, 0, 300)
    assert [int(v) for v in ctr] == seq
    # any window of the stream can be drawn on its own
    assert [int(v) for v in P.splitmix64(seed, 117, 50)] == seq[117:167]


def test_uniform_range_and_moments():
    u = P.uniform(7, (200_000,), -0.1, 0.1)
    assert u.min() >= -0.1 and u.max() < 0.1
    assert abs(u.mean()) < 1e-3
    assert abs(u.var() - 0.2**2 / 12) < 1e-4


def test_normal_moments():
    z = P.normal(21, (200_000,))
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01


def test_torch_form_bitwise_equal_to_numpy():
    torch = pytest.importorskip("torch")
    a = P.pfc_initial_field(3, (6, 5, 8), -0.3)
    b = P.pfc_initial_field_torch(3, (6, 5, 8), -0.3, torch.float64, "cpu").numpy()
    assert np.array_equal(a, b)
    b32 = P.pfc_initial_field_torch(3, (6, 5, 8), -0.3, torch.float32, "cpu").numpy()
    assert np.array_equal(a.astype(np.float32), b32)
    # chunk boundaries do not change values
    c = P.uniform_torch(9, (1000,), -1, 1, torch.float64, "cpu", chunk=97).numpy()
    assert np.array_equal(c, P.uniform(9, (1000,), -1, 1))
