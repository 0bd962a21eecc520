"""The indicator's division-free shortcut (eq. calc-blending-factor) decides nothing
differently from the division it skips: wherever |s_n - s_h| < fl(0.99 tau_S) * den, the
rounded quotient lies below tau_S, so tau_A (r - tau_S) is negative and the ramp clamps
to 0.  Checked here in IEEE double arithmetic (the kernel's), by brute force over
magnitudes, near-boundary cases and the parameter guards; no GPU."""
import numpy as np
import pytest


def quick_bound(tau_A, tau_S):
    # the host-side value the library passes to the analysis (0: no shortcut)
    ok = tau_A >= 0.0 and tau_A <= np.finfo(np.float64).max and tau_S > 0.0
    return np.float64(0.99) * np.float64(tau_S) if ok else np.float64(0.0)


def ramp(d, den, tau_A, tau_S):
    r = d / den
    x = np.float64(tau_A) * (r - np.float64(tau_S))
    return np.where(x < 0.0, 0.0, np.where(x > 1.0, 1.0, x))


@pytest.mark.parametrize("tau_A,tau_S", [(100.0, 0.05), (1.0, 1e-3), (1e6, 0.5), (0.0, 0.05), (3.0, 1e-12)])
def test_quick_bound_implies_zero_ramp(tau_A, tau_S):
    rng = np.random.default_rng(11)
    q = quick_bound(tau_A, tau_S)
    n = 400_000
    den = np.exp(rng.uniform(np.log(1e-12), np.log(1e12), n))
    # d spread around the bound: relative positions within +-1e-3 of q den, and far below
    rel = np.concatenate([rng.uniform(0.999, 1.001, n // 2), rng.uniform(0.0, 1.0, n - n // 2)])
    d = rel * q * den
    # also the doubles adjacent to the bound itself
    b = q * den[:1000]
    d = np.concatenate([d, np.nextafter(b, 0.0), b, np.nextafter(b, np.inf)])
    den = np.concatenate([den, den[:1000], den[:1000], den[:1000]])
    taken = d < q * den
    assert taken.sum() > n // 3
    r = d[taken] / den[taken]
    assert np.all(r < tau_S)
    assert np.all(ramp(d[taken], den[taken], tau_A, tau_S) == 0.0)


@pytest.mark.parametrize("tau_A,tau_S", [(-1.0, 0.05), (np.inf, 0.05), (np.nan, 0.05), (100.0, 0.0),
                                         (100.0, -0.05), (100.0, np.nan)])
def test_quick_bound_guards(tau_A, tau_S):
    """Outside its argument's assumptions (a negative or infinite amplification, a
    non-positive threshold) the bound is 0, which no |difference| >= 0 falls below."""
    q = quick_bound(tau_A, tau_S)
    assert q == 0.0
    d = np.array([0.0, 1e-300, 1.0])
    assert not np.any(d < q * np.array([1.0, 1.0, 1.0]))
