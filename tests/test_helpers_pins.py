"""The parity gates of the GPU tests (tests/helpers.err) are pinned here on
the CPU: the per-step error never reads below the stacked one, and one wrong
step in a long horizon is not diluted by the number of steps."""
import numpy as np

from tests.helpers import err, rel, step_rel


def test_one_wrong_step_is_not_diluted():
    rng = np.random.default_rng(0)
    T = 100_000
    b = rng.standard_normal((T, 4))
    a = b.copy()
    a[T // 2] *= 1.0 + 1e-6  # one step off by 1e-6 of its size
    assert rel(a, b) < 1e-8  # the stacked norm hides it ...
    assert step_rel(a, b) > 5e-7  # ... the per-step error does not
    assert err(a, b) == step_rel(a, b)


def test_step_rel_bounds_rel_from_above_for_even_steps():
    rng = np.random.default_rng(1)
    for shape in [(1, 3), (7, 2, 2), (50, 5)]:
        b = np.ones(shape)  # every step of the same size: the RMS size
        a = b + 1e-9 * rng.standard_normal(shape)
        assert step_rel(a, b) >= rel(a, b)


def test_large_step_is_held_to_its_own_size():
    b = np.full((1000, 2), 1e-3)
    b[0] = 10.0  # one step far above the RMS size
    a = b.copy()
    a[0] *= 1.0 + 1e-7
    assert abs(step_rel(a, b) - 1e-7) < 1e-12
    a = b.copy()
    a[500] *= 1.0 + 1e-3  # a small step off by 1e-3 of its size
    assert step_rel(a, b) > 2e-6  # measured against the RMS step, not hidden


def test_zero_reference_is_absolute():
    b = np.zeros((10, 3))
    a = b.copy()
    a[3, 1] = 2e-12
    assert step_rel(a, b) == 2e-12
    assert rel(a, b) == 2e-12
