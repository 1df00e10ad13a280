"""Pins of the oracle's not-a-knot cubic spline (Sec. II.A: tridiagonal cubic
spline of each sparse function, SciPy-style) against independent references."""
import numpy as np
import pytest
from scipy.interpolate import CubicSpline


def _logknots(n, a=2e-5, b=3e-2):
    return np.geomspace(a, b, n)


@pytest.mark.parametrize("n", [4, 5, 17, 256])
def test_matches_scipy_not_a_knot(oracle, n):
    rng = np.random.default_rng(n)
    x = np.sort(rng.uniform(0.0, 10.0, n))
    x = np.unique(x)
    y = rng.standard_normal(x.size)
    coef = oracle.spline_coeffs(x, y)
    ref = CubicSpline(x, y, bc_type="not-a-knot")
    # scipy stores c[k, i] for (x - x_i)^(3-k); compare each term's
    # contribution over its interval, c_k h^k, against the data scale
    ours = coef[:, ::-1].T
    hpow = np.diff(x)[None, :] ** np.arange(3, -1, -1)[:, None]
    assert np.max(np.abs(ours - ref.c) * hpow) < 1e-11 * np.abs(y).max()
    xq = np.concatenate([x, rng.uniform(x[0], x[-1], 1000)])
    yq = oracle.spline_eval(x, coef, xq)
    assert np.max(np.abs(yq - ref(xq))) < 1e-11 * np.abs(y).max()


def test_matches_scipy_on_log_knots_and_chirp_phase(oracle):
    # the sparse grids of the method: 256 log-spaced knots, phase values ~1e7 rad
    x = _logknots(256)
    y = 2 * np.pi * 3.15e7 * x + 1e3 * x ** (-5.0 / 3.0) * 1e-4
    coef = oracle.spline_coeffs(x, y)
    ref = CubicSpline(x, y, bc_type="not-a-knot")
    xq = np.geomspace(x[0], x[-1], 5000)
    err = np.abs(oracle.spline_eval(x, coef, xq) - ref(xq))
    assert err.max() < 1e-14 * np.abs(y).max() * 64


@pytest.mark.parametrize("n", [4, 9, 256])
def test_reproduces_cubics(oracle, n):
    x = _logknots(n, 1.0, 7.0)
    p = np.array([0.3, -1.7, 2.2, -0.45])  # c0 + c1 x + c2 x^2 + c3 x^3
    y = np.polyval(p[::-1], x)
    coef = oracle.spline_coeffs(x, y)
    xq = np.linspace(1.0, 7.0, 3001)
    yq = oracle.spline_eval(x, coef, xq)
    assert np.max(np.abs(yq - np.polyval(p[::-1], xq))) < 1e-12 * np.abs(y).max()


def test_tridiagonal_solve_matches_dense_solve(oracle):
    rng = np.random.default_rng(3)
    n = 64
    sub = rng.uniform(0.1, 1.0, n)
    sup = rng.uniform(0.1, 1.0, n)
    dia = sub + sup + rng.uniform(0.5, 2.0, n)
    rhs = rng.standard_normal(n)
    A = np.diag(dia) + np.diag(sub[1:], -1) + np.diag(sup[:-1], 1)
    x = oracle.tridiag(sub, dia, sup, rhs)
    assert np.allclose(x, np.linalg.solve(A, rhs), rtol=1e-13, atol=1e-13)


def test_interval_lookup_is_largest_knot_below(oracle):
    # piecewise-constant data would hide the interval; use coefficients that
    # tag each interval with its index and evaluate at dx = 0
    n = 33
    x = np.geomspace(1e-4, 1e-1, n)
    coef = np.zeros((n - 1, 4))
    coef[:, 0] = np.arange(n - 1)
    rng = np.random.default_rng(5)
    xq = np.concatenate([x, rng.uniform(x[0], x[-1], 2000)])
    got = oracle.spline_eval(x, coef, xq)
    brute = np.array([max(i for i in range(n - 1) if x[i] <= v) for v in xq])
    assert np.array_equal(got.astype(int), brute)


def test_rejects_bad_knots(oracle):
    with pytest.raises(ValueError):
        oracle.spline_coeffs(np.array([0.0, 1.0, 1.0, 2.0]), np.zeros(4))
    with pytest.raises(ValueError):
        oracle.spline_coeffs(np.array([0.0, 1.0, 2.0]), np.zeros(3))


def test_loglike_converges_at_fourth_order_in_knot_spacing(oracle):
    """Sec. II.A represents each function on a sparse grid (about 2^10 points)
    and splines it to the data bins.  A cubic spline with not-a-knot ends
    interpolates a smooth function with error O(h^4), so ln L at n_s knots
    approaches its dense-knot limit with the error falling about 16-fold per
    doubling of n_s; a lower-order end condition or interval lookup would
    show a smaller ratio."""
    from paper_2005_01827_amd import inputs
    w = inputs.small_config(4)
    g = w.grid
    psd = inputs.psd_aet(g.freqs)
    d = oracle.template(w.injection, g, w.modes, 2048, w.t0) + inputs.noise(g, psd, 5)
    ref = oracle.loglike(w.walkers, g, d, psd, w.modes, 2048, w.t0)[:, 0]
    errs = [np.abs(oracle.loglike(w.walkers, g, d, psd, w.modes, ns, w.t0)[:, 0] - ref).max()
            for ns in (128, 256, 512, 1024)]
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all((ratios > 12) & (ratios < 22)), ratios
