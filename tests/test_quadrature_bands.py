"""The mixed kernel replaces the closed-form field of a source segment by an
n-point Gauss-Legendre rule along the source when the target lies outside a
band around the source midpoint: 30 source lengths for 2 points, 6 for 3.
This checks, on the FP64 oracle, that both rules stay below 2e-7 relative
error there (well under the mixed path's 1e-4 tolerance), at many random
orientations and at the band edge where the error is largest."""
import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("n,band", [(2, 30.0), (3, 6.0)])
def test_source_rule_error_outside_band(n, band):
    rng = np.random.default_rng(11)
    worst = 0.0
    for _ in range(300):
        L = rng.uniform(5.0, 200.0)
        t = rng.normal(size=3)
        t /= np.linalg.norm(t)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        b = rng.normal(size=3)
        b /= np.linalg.norm(b)
        x1, x2 = np.zeros(3), L * t
        x = 0.5 * L * t + band * L * d
        s = O.segment_stress(x, x1, x2, b, 1.0, 0.34, 1.0)
        q = O.segment_stress_quad(x, x1, x2, b, 1.0, 0.34, 1.0, n, 1)
        worst = max(worst, np.linalg.norm(q - s) / np.linalg.norm(s))
    assert worst < 2e-7, worst


def test_three_point_rule_fails_inside_its_band():
    """The band is not wider than needed by orders of magnitude: at 3 source
    lengths the 3-point rule is already off by more than 1e-6."""
    rng = np.random.default_rng(12)
    worst = 0.0
    for _ in range(200):
        L = 50.0
        t = rng.normal(size=3)
        t /= np.linalg.norm(t)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        b = rng.normal(size=3)
        b /= np.linalg.norm(b)
        x = 0.5 * L * t + 3.0 * L * d
        s = O.segment_stress(x, np.zeros(3), L * t, b, 1.0, 0.34, 1.0)
        q = O.segment_stress_quad(x, np.zeros(3), L * t, b, 1.0, 0.34, 1.0, 3, 1)
        worst = max(worst, np.linalg.norm(q - s) / np.linalg.norm(s))
    assert worst > 1e-6, worst
