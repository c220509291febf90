"""The synthetic generators draw what their docstrings state (no method arithmetic).

Gaussians on the Swiss roll: the inverse of the spiral's arc length is exact,
every point lies on the rotated roll at the intrinsic coordinates it was
drawn at, the means sit inside the shrunken strip, labels count per_dist.
"""
import numpy as np

import synth


def test_roll_arclength_inverse():
    u = np.linspace(0.05, 25.0, 400)
    np.testing.assert_allclose(synth._roll_param_of_arclength(synth._roll_arclength(u)), u, rtol=1e-12)
    # arc length of the spiral (u cos u, u sin u) by quadrature of sqrt(1 + u^2)
    from scipy.integrate import quad
    for a, b in [(1.0, 2.0), (4.7, 14.1)]:
        ref = quad(lambda x: np.sqrt(1 + x * x), a, b)[0]
        assert abs(synth._roll_arclength(b) - synth._roll_arclength(a) - ref) < 1e-10


def test_gaussians_on_swiss_roll_lie_on_the_roll():
    X, lab, means = synth.gaussians_on_swiss_roll(6, 200, dim=10, sigma=2.0, workload=9)
    assert X.shape == (1200, 10) and X.dtype == np.float32
    assert np.all(np.bincount(lab) == 200)
    s_lo, s_hi = synth._roll_arclength(np.array([1.5 * np.pi, 4.5 * np.pi]))
    assert np.all(means[:, 0] >= s_lo + 4.0) and np.all(means[:, 0] <= s_hi - 4.0)
    assert np.all(means[:, 1] >= 4.0) and np.all(means[:, 1] <= 17.0)
    # undo the rotation (orthonormal columns of the lift), then check the spiral
    q, _ = np.linalg.qr(np.random.default_rng(synth.seed_for(9, 1)).standard_normal((10, 3)))
    R = X.astype(np.float64) @ q                     # (x, h, z) in R^3
    u = np.hypot(R[:, 0], R[:, 2])                   # radius of the spiral = u
    np.testing.assert_allclose(R[:, 0], u * np.cos(u), atol=2e-4 * u.max())
    np.testing.assert_allclose(R[:, 2], u * np.sin(u), atol=2e-4 * u.max())
    # intrinsic coordinates scatter around their own means
    s = synth._roll_arclength(u)
    for i in range(6):
        m = lab == i
        assert abs(s[m].mean() - means[i, 0]) < 0.5 and abs(R[m, 1].mean() - means[i, 1]) < 0.5
