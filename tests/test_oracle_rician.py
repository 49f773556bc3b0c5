"""Pins for the Rician data term (App. D.3.3) of the oracle: the Bessel
functions against scipy's independent implementation and their limits, the
likelihood's normalisation, the zero-mean score, and central differences of
f, grad f and its Hessian."""
import numpy as np
import pytest
import scipy.special as sp

from oracle import bessel, operators as O


def test_scaled_bessel_against_scipy():
    t = np.concatenate([np.linspace(0.0, 80.0, 8001), np.geomspace(1e-9, 1e5, 3000),
                        [29.999999, 30.0, 30.000001]])
    i0, i1 = bessel.i0_i1_scaled(t)
    np.testing.assert_allclose(i0, sp.i0e(t), rtol=5e-15, atol=0)
    np.testing.assert_allclose(i1, sp.i1e(t), rtol=5e-15, atol=1e-300)


def test_ratio_is_odd_and_has_its_limits():
    t = np.geomspace(1e-6, 1e-2, 20)
    b = bessel.ratio(t)
    np.testing.assert_allclose(b, t / 2 - t ** 3 / 16 + t ** 5 / 96, rtol=1e-12)
    np.testing.assert_allclose(bessel.ratio(-t), -b, rtol=0, atol=0)
    big = np.geomspace(1e3, 1e6, 10)
    err = np.abs(bessel.ratio(big) - (1 - 1 / (2 * big) - 1 / (8 * big ** 2)))
    assert np.all(err <= 2 / big ** 3 + 2e-16)
    assert bessel.ratio(np.array([0.0]))[0] == 0.0


def test_log_i0_derivative_is_the_ratio():
    t = np.array([-40.0, -3.0, -0.2, 0.1, 1.0, 7.5, 29.9, 30.1, 55.0, 400.0])
    h = 1e-5
    fd = (bessel.log_i0(t + h) - bessel.log_i0(t - h)) / (2 * h)
    np.testing.assert_allclose(fd, bessel.ratio(t), rtol=1e-8, atol=1e-10)
    fd2 = (bessel.ratio(t + h) - bessel.ratio(t - h)) / (2 * h)
    np.testing.assert_allclose(fd2, bessel.ratio_derivative(t), rtol=1e-6, atol=1e-9)
    assert bessel.ratio_derivative(np.array([0.0]))[0] == 0.5


@pytest.mark.parametrize("x", [0.0, 0.05, 0.3, 0.9])
def test_likelihood_integrates_to_one(x):
    """p(y|x) = y/s^2 exp(-(x^2 + y^2)/(2 s^2)) I_0(x y / s^2) is a density in y,
    with f = -log p up to a constant: exp(-f) y/s^2 exp(-y^2/(2 s^2)) integrates to 1."""
    s = 25.5 / 255.0
    yy = np.linspace(0.0, x + 12 * s, 200001)
    op = O.Operator("rician", sigma=s)
    fvals = op.f(np.full((1, 1, 1, yy.size), x), yy.reshape(1, 1, 1, -1))  # summed: use per-point
    per_point = x * x / (2 * s * s) - bessel.log_i0(x * yy / (s * s))
    assert abs(fvals[0] - per_point.sum()) < 1e-9 * abs(per_point.sum()) + 1e-9
    dens = yy / s ** 2 * np.exp(-yy ** 2 / (2 * s * s) - per_point)
    integral = np.trapezoid(dens, yy)
    assert abs(integral - 1.0) < 1e-8


def test_score_has_zero_mean_at_the_true_value():
    """E_y[grad_x f(x, y)] = 0 at the true x (the score of a likelihood)."""
    rng = np.random.default_rng(7)
    s = 12.75 / 255.0
    op = O.Operator("rician", sigma=s)
    for x in (0.02, 0.2, 0.7):
        n = 400000
        y = np.sqrt((x + s * rng.standard_normal(n)) ** 2 + (s * rng.standard_normal(n)) ** 2)
        g = op.grad_f(np.full((1, 1, 1, n), x), y.reshape(1, 1, 1, -1))[0, 0, 0]
        # standard error of the mean score is about 1 / (s sqrt(n))
        assert abs(g.mean()) < 5.0 / (s * np.sqrt(n)), (x, g.mean())
        # and the score at a wrong x is far from zero
        gw = op.grad_f(np.full((1, 1, 1, n), x + 0.1), y.reshape(1, 1, 1, -1))[0, 0, 0]
        assert abs(gw.mean()) > 50.0 / (s * np.sqrt(n))


def test_gradient_and_hessian_by_central_differences(rng):
    s = 25.5 / 255.0
    op = O.Operator("rician", sigma=s)
    x = rng.uniform(-0.2, 1.1, (2, 3, 4, 5))
    y = np.abs(rng.uniform(0.0, 1.2, x.shape))
    w = rng.standard_normal(x.shape)
    h = 1e-6
    fd = (op.f(x + h * w, y) - op.f(x - h * w, y)) / (2 * h)
    np.testing.assert_allclose(fd, np.sum(op.grad_f(x, y) * w, axis=(1, 2, 3)), rtol=1e-7)
    fd2 = (op.grad_f(x + h * w, y) - op.grad_f(x - h * w, y)) / (2 * h)
    np.testing.assert_allclose(fd2, op.hess_f(x, y, w), rtol=1e-5, atol=1e-4)


def test_zero_measurement_is_a_quadratic():
    s = 0.1
    op = O.Operator("rician", sigma=s)
    x = np.linspace(-1, 1, 24).reshape(1, 2, 3, 4)
    y = np.zeros_like(x)
    np.testing.assert_allclose(op.grad_f(x, y), x / s ** 2, rtol=1e-15)
    np.testing.assert_allclose(op.f(x, y), [np.sum(x * x) / (2 * s * s)], rtol=1e-15)
