"""The map from the reverse raster pass's slot moments to the 2D gradient.

The GPU reverse pass sums, per record, the moments of gp = dL/dp over the
pixel offsets d = pixel - mean2d (gp dx, gp dy, gp dx^2, gp dx dy, gp dy^2),
where p = -(A dx^2 + 2 B dx dy + C dy^2) / 2 is the exponent of the
Gaussian's alpha (Sec. 3.2); tests/parity.slot_grad2d turns them into the 2D
gradient the oracle reports.  Checked here against central differences of
sum_pixels gp * p(pixel; mean, A, B, C) in every one of the five geometric
parameters, on random conics, pixels and weights."""
import numpy as np

from parity import slot_grad2d


def exponent(px, py, mx, my, A, B, C):
    dx, dy = px - mx, py - my
    return -0.5 * (A * dx * dx + 2.0 * B * dx * dy + C * dy * dy)


def test_slot_moments_give_the_2d_gradient():
    rng = np.random.default_rng(7)
    for _ in range(20):
        # a positive-definite conic, a mean, pixels around it and weights gp
        L = rng.normal(size=(2, 2))
        Q = L @ L.T + 0.1 * np.eye(2)
        A, B, C = Q[0, 0], Q[0, 1], Q[1, 1]
        mx, my = rng.uniform(-50, 50, size=2)
        px = mx + rng.normal(scale=3.0, size=40)
        py = my + rng.normal(scale=3.0, size=40)
        gp = rng.normal(size=40)
        dx, dy = px - mx, py - my
        slots = np.zeros((1, 16))
        slots[0, :5] = [np.sum(gp * dx), np.sum(gp * dy), np.sum(gp * dx * dx), np.sum(gp * dx * dy),
                        np.sum(gp * dy * dy)]
        slots[0, 5:9] = rng.normal(size=4)  # opacity and colour terms pass through
        got = slot_grad2d(slots, np.array([[A], [B], [C]]))[0]

        def f(theta):
            return np.sum(gp * exponent(px, py, *theta))

        theta = np.array([mx, my, A, B, C])
        h = 1e-5
        want = np.empty(5)
        for k in range(5):
            e = np.zeros(5)
            e[k] = h
            want[k] = (f(theta + e) - f(theta - e)) / (2 * h)
        np.testing.assert_allclose(got[:5], want, rtol=1e-6, atol=1e-6 * np.abs(want).max())
        np.testing.assert_array_equal(got[5:9], slots[0, 5:9])
