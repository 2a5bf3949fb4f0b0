"""The helper that compares two converged results (agreement.py) on
synthetic cases: a difference along the rank-mass direction up to twice the
bar passes, any other difference above the bar fails."""
import numpy as np

from agreement import agree


def _ref(n=500, seed=3):
    r = np.random.default_rng(seed).pareto(1.5, n) + 1.0
    return r / r.sum()


def test_mass_direction_difference_up_to_twice_the_bar():
    ref = _ref()
    c = 0.9e-9 / ref.max()
    a, b = ref * (1 + c), ref * (1 - c)  # each 0.9e-9 from ref, 1.8e-9 apart
    ok, perp, whole = agree(a, b, ref, 1e-9)
    assert ok and perp < 1e-15 and 1.7e-9 < whole < 1.9e-9
    # beyond twice the bar the whole difference fails
    c = 1.1e-9 / ref.max()
    assert not agree(ref * (1 + c), ref * (1 - c), ref, 1e-9)[0]


def test_other_differences_above_the_bar_fail():
    ref = _ref()
    a = ref.copy()
    b = ref.copy()
    b[7] += 1.5e-9  # one rank: not along the mass direction
    ok, perp, whole = agree(a, b, ref, 1e-9)
    assert not ok and perp > 1e-9
    b[7] = ref[7] + 0.5e-9
    assert agree(a, b, ref, 1e-9)[0]


def test_relative_bar():
    ref = _ref()
    b = ref * (1 + 1e-7)
    ok, perp, whole = agree(ref, b, ref, 1e-6, relative=True)
    assert ok and abs(whole - 1e-7) < 1e-9
    b2 = ref.copy()
    b2[0] += 3e-6 * ref.max()
    assert not agree(ref, b2, ref, 1e-6, relative=True)[0]
