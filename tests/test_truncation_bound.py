"""The covariance generation stops its quadrature past an upper bound of the
root t* of F(t) = x (cosh t - 1) - g t - 45 (g = |nu| + 1): two acosh
iterates t1 <= t2 <= t* and the bound t2 + g (t2 - t1) / (45 - g), which holds
because F' >= 45 - g beyond t2.  The inequality is checked here against the
root found by bisection over the range of x and nu the kernels see."""
import math

import numpy as np


def acosh_ge1(y):
    return math.log(y + math.sqrt((y - 1.0) * (y + 1.0)))


def bound(x, g):
    t1 = acosh_ge1(1.0 + 45.0 / x)
    t2 = acosh_ge1(1.0 + (45.0 + g * t1) / x)
    return t1, t2, t2 + g * (t2 - t1) / (45.0 - g)


def root(x, g):
    f = lambda t: x * (math.cosh(t) - 1.0) - g * t - 45.0
    lo, hi = 0.0, 1.0
    while f(hi) < 0:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) < 0:
            lo = mid
        else:
            hi = mid
    return hi


def test_bound_is_above_the_root_and_tight():
    gen = np.random.default_rng(11)
    xs = 10.0 ** gen.uniform(-8, 3, 400)
    gs = 1.0 + gen.uniform(0.0, 6.0, 400)       # nu up to 6
    for x, g in zip(xs, gs):
        t1, t2, tb = bound(x, g)
        ts = root(x, g)
        assert t1 <= t2 <= ts * (1 + 1e-12)
        assert tb >= ts * (1 - 1e-12), (x, g, tb, ts)
        assert tb - ts <= 0.25                  # about one node of the coarsest step (0.2)


def test_integrand_is_negligible_past_the_bound():
    """exp(-x (cosh t - 1)) cosh(nu t) at the bound is below e^-45 (times the
    cosh/exp ratio bound used by F), for the same sample."""
    gen = np.random.default_rng(12)
    for _ in range(200):
        x = 10.0 ** gen.uniform(-6, 3)
        nu = gen.uniform(0.0, 5.0)
        _, _, tb = bound(x, nu + 1.0)
        log_val = -x * (math.cosh(tb) - 1.0) + nu * tb + math.log1p(math.exp(-2 * nu * tb)) - math.log(2)
        assert log_val <= -45.0 + 1e-9
