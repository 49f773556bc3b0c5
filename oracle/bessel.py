"""Modified Bessel functions I_0, I_1 of the first kind and the ratio
B(t) = I_1(t) / I_0(t) of the Rician data term (App. D.3.3), float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Both functions are evaluated from their textbook definitions
(Abramowitz & Stegun, Handbook of Mathematical Functions, 9.6.10 and 9.7.1):
  * t <= T_SWITCH: the power series
        I_nu(t) = sum_{k>=0} (t/2)^(2k+nu) / (k! (k+nu)!),
    summed term by term (all terms are positive, so there is no cancellation);
  * t >  T_SWITCH: the large-argument expansion
        I_nu(t) = e^t / sqrt(2 pi t) * sum_k (-1)^k a_k(nu) / t^k,
        a_k(nu) = prod_{j=1..k} (4 nu^2 - (2j - 1)^2) / (k! 8^k),
    summed while its terms decrease; its truncation error is below the
    smallest term, about e^(-2t), far under float64 rounding for t > 30.
Values are returned scaled by e^(-t) so that large arguments do not overflow.
I_0 is even and I_1 odd, so B is odd and log I_0 even.

Pins: scipy.special.i0e / i1e (an independent implementation), the
derivative identity d/dt log I_0(t) = B(t) by central differences, and
B(t) -> t/2 as t -> 0, B(t) -> 1 - 1/(2t) as t -> inf
(tests/test_oracle_rician.py).
"""
import numpy as np

T_SWITCH = 30.0
SERIES_TERMS = 120       # (t/2)^2k / (k!)^2 is below 1e-18 of the sum by k = 120 for t <= 30
ASYMP_TERMS = 60         # terms decrease for k < 2t; 60 < 2 * T_SWITCH


def _series(t, nu):
    """e^{-t} I_nu(t) for 0 <= t <= T_SWITCH by the power series."""
    q = (0.5 * t) ** 2
    term = np.ones_like(t) if nu == 0 else 0.5 * t
    total = term.copy()
    for k in range(1, SERIES_TERMS):
        term = term * q / (k * (k + nu))
        total = total + term
    return total * np.exp(-t)


def _asymptotic(t, nu):
    """e^{-t} I_nu(t) for t > T_SWITCH by the large-argument expansion."""
    mu = 4.0 * nu * nu
    term = np.ones_like(t)
    total = term.copy()
    for k in range(1, ASYMP_TERMS):
        term = -term * (mu - (2 * k - 1) ** 2) / (k * 8.0 * t)
        total = total + term
    return total / np.sqrt(2.0 * np.pi * t)


def i0_i1_scaled(t):
    """(e^{-|t|} I_0(|t|), e^{-|t|} I_1(|t|)) elementwise."""
    a = np.abs(np.asarray(t, dtype=np.float64))
    small = a <= T_SWITCH
    i0 = np.empty_like(a)
    i1 = np.empty_like(a)
    i0[small] = _series(a[small], 0)
    i1[small] = _series(a[small], 1)
    i0[~small] = _asymptotic(a[~small], 0)
    i1[~small] = _asymptotic(a[~small], 1)
    return i0, i1


def ratio(t):
    """B(t) = I_1(t) / I_0(t) (odd in t)."""
    t = np.asarray(t, dtype=np.float64)
    i0, i1 = i0_i1_scaled(t)
    return np.sign(t) * i1 / i0


def log_i0(t):
    """log I_0(t) = |t| + log(e^{-|t|} I_0(|t|))."""
    t = np.asarray(t, dtype=np.float64)
    i0, _ = i0_i1_scaled(t)
    return np.abs(t) + np.log(i0)


def ratio_derivative(t):
    """B'(t) = 1 - B(t)/t - B(t)^2 (from I_0' = I_1, I_1' = I_0 - I_1/t);
    B'(0) = 1/2."""
    t = np.asarray(t, dtype=np.float64)
    b = ratio(t)
    with np.errstate(divide="ignore", invalid="ignore"):
        bt = np.where(t != 0.0, b / np.where(t != 0.0, t, 1.0), 0.5)
    return 1.0 - bt - b * b
