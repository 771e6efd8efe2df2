"""The comparison helper of the parity tests catches one wrong small entry that the
norm-wise check alone lets through."""
import numpy as np
import pytest

from parity import assert_parity, max_entry_err, rel


def test_entrywise_check_catches_a_small_wrong_entry():
    rng = np.random.default_rng(0)
    b = rng.standard_normal(10_000)
    a = b.copy()
    a[17] += 50e-6  # one entry off by 5e-5 of the largest entry
    assert rel(a, b) < 1e-6  # hidden under the norm of the others
    assert max_entry_err(a, b) > 1e-5
    with pytest.raises(AssertionError):
        assert_parity(a, b, 1e-6)


def test_accepts_rounding_level_differences():
    rng = np.random.default_rng(1)
    b = rng.standard_normal(1000)
    a = b * (1 + 1e-15 * rng.standard_normal(1000))
    r, m = assert_parity(a, b, 1e-13)
    assert r < 1e-13 and m < 1e-13


def test_rejects_non_finite_and_shape_mismatch():
    b = np.ones(4)
    with pytest.raises(AssertionError):
        assert_parity(np.array([1.0, np.nan, 1.0, 1.0]), b, 1e-3)
    with pytest.raises(AssertionError):
        assert_parity(np.ones(3), b, 1e-3)
