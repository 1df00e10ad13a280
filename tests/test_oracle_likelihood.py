"""Pins of the oracle's dense stage and likelihood: Eq. NLL, Eq. innerprod
discretised on f_k = k df, Eq. innerprodsum over A, E, T, and the noise model
of Eq. noise_gen.  Also the seeded input generators (D_L(z), PSD, noise)."""
import math
import os

import numpy as np
import pytest
from scipy.interpolate import CubicSpline

from paper_2005_01827_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def small():
    w = inputs.small_config(4)
    psd = inputs.psd_aet(w.grid.freqs)
    return w, psd


def test_noiseless_self_injection_is_exactly_zero(oracle, small):
    w, psd = small
    h = oracle.template(w.injection, w.grid, w.modes, w.ns, w.t0)
    out = oracle.loglike(w.injection[None], w.grid, h, psd, w.modes, w.ns, w.t0)
    assert out[0, 0] == 0.0
    assert np.all(out[0, 1:4] == out[0, 4:7])


def test_nll_two_forms_agree(oracle, small):
    """-ln L = 1/2 <d-h|d-h> = 1/2 (<d|d> + <h|h> - 2 <d|h>)."""
    w, psd = small
    g = w.grid
    d = oracle.template(w.injection, g, w.modes, w.ns, w.t0) + inputs.noise(g, psd, 11)
    out = oracle.loglike(w.walkers, g, d, psd, w.modes, w.ns, w.t0)
    dd = sum(math.fsum(4 * g.df * np.abs(d[c]) ** 2 / psd[c]) for c in range(3))
    other = -0.5 * (dd + out[:, 4:7].sum(1) - 2 * out[:, 1:4].sum(1))
    assert np.allclose(out[:, 0], other, rtol=1e-10, atol=0)


def test_inner_products_against_brute_force_summation(oracle, small):
    """<d|h>_c and <h|h>_c against exact (fsum) summation of the oracle's own
    template: checks the discretised Eq. innerprod and the channel sum."""
    w, psd = small
    g = w.grid
    d = inputs.noise(g, psd, 12)
    th = w.walkers[1]
    h = oracle.template(th, g, w.modes, w.ns, w.t0)
    out = oracle.loglike(th[None], g, d, psd, w.modes, w.ns, w.t0)[0]
    for c in range(3):
        wgt = 4 * g.df / psd[c]
        dh = math.fsum((d[c].real * h[c].real + d[c].imag * h[c].imag) * wgt)
        hh = math.fsum((h[c].real ** 2 + h[c].imag ** 2) * wgt)
        # symmetric form of Eq. innerprod: 2 int (a b* + a* b)/S df
        sym = math.fsum((2 * (d[c] * np.conj(h[c]) + np.conj(d[c]) * h[c]).real / psd[c]) * g.df)
        assert abs(out[1 + c] - dh) <= 1e-10 * math.sqrt(hh) + 1e-12 * abs(dh)
        assert abs(out[4 + c] - hh) <= 1e-12 * hh
        assert abs(dh - sym) <= 1e-10 * math.sqrt(hh)
        assert hh >= 0.0


def test_template_against_independent_spline_library(oracle, small):
    """Dense template = sum over modes of S_T S_A exp(i S_phi), rebuilt from
    the oracle's sparse knot values with scipy's not-a-knot CubicSpline."""
    w, psd = small
    g = w.grid
    th = w.walkers[2]
    sp = oracle.sparse(th, g, w.modes, w.ns, w.t0)
    h = oracle.template(th, g, w.modes, w.ns, w.t0)
    k = g.k0 + np.arange(g.n)
    f = k * g.df
    ref = np.zeros((3, g.n), complex)
    for im in range(len(w.modes)):
        active, klo, khi, _ = sp["band"][im]
        if not active:
            continue
        sel = (k >= klo) & (k <= khi)
        x = sp["f"][im]
        val = [CubicSpline(x, sp["fn"][im, q], bc_type="not-a-knot")(f[sel]) for q in range(8)]
        wave = val[0] * np.exp(1j * val[1])
        for c in range(3):
            ref[c, sel] += (val[2 + 2 * c] + 1j * val[3 + 2 * c]) * wave
    scale = np.abs(ref).max()
    # phases reach ~1e6 rad: two spline codes agree to ~1e-9 rad there
    assert np.max(np.abs(h - ref)) < 1e-7 * scale


def test_hh_scales_as_inverse_distance_squared(oracle, small):
    w, psd = small
    th = w.walkers[0].copy()
    d = np.zeros((3, w.grid.n), complex)
    a = oracle.loglike(th[None], w.grid, d, psd, w.modes, w.ns, w.t0)[0]
    th[4] *= 2.5
    b = oracle.loglike(th[None], w.grid, d, psd, w.modes, w.ns, w.t0)[0]
    assert np.allclose(a[4:7] / b[4:7], 2.5 ** 2, rtol=1e-12)


def test_phi_ref_periodicity(oracle, small):
    w, psd = small
    g = w.grid
    d = oracle.template(w.injection, g, w.modes, w.ns, w.t0) + inputs.noise(g, psd, 13)
    th = w.walkers[3].copy()
    th2 = th.copy()
    th2[5] += 2 * math.pi
    a = oracle.loglike(np.stack([th, th2]), g, d, psd, w.modes, w.ns, w.t0)
    assert abs(a[0, 0] - a[1, 0]) < 1e-9 * abs(a[0, 0])
    # a (2,2)-only template repeats after pi
    th3 = th.copy()
    th3[5] += math.pi
    b = oracle.loglike(np.stack([th, th3]), g, d, psd, [(2, 2)], w.ns, w.t0)
    assert abs(b[0, 0] - b[1, 0]) < 1e-9 * abs(b[0, 0])
    c = oracle.loglike(np.stack([th, th3]), g, d, psd, w.modes, w.ns, w.t0)
    assert abs(c[0, 0] - c[1, 0]) > 1e-6 * abs(c[0, 0])


def test_invalid_walkers_get_minus_inf(oracle, small):
    w, psd = small
    th = np.repeat(w.injection[None], 4, axis=0)
    th[1, 1] = 1.5
    th[2, 2] = -1.0
    th[3, 4] = float("nan")
    d = np.zeros((3, w.grid.n), complex)
    out = oracle.loglike(th, w.grid, d, psd, w.modes, w.ns, w.t0)
    assert np.isfinite(out[0, 0]) and np.all(np.isneginf(out[1:, 0]))


def test_noise_chi_square_and_overlap(oracle, small):
    """Eq. noise_gen with the one-sided reading: <n|n>_c ~ chi^2 with mean 2
    per bin; <n|h> ~ N(0, <h|h>^(1/2))."""
    w, psd = small
    g = w.grid
    n = inputs.noise(g, psd, 99)
    for c in range(3):
        nn = np.sum(4 * g.df * np.abs(n[c]) ** 2 / psd[c])
        assert abs(nn - 2 * g.n) < 5 * 2 * math.sqrt(g.n)
    th = w.injection
    z = []
    for seed in range(48):
        d = inputs.noise(g, psd, 1000 + seed)
        out = oracle.loglike(th[None], g, d, psd, [(2, 2)], w.ns, w.t0)[0]
        z.append(out[1:4].sum() / math.sqrt(out[4:7].sum()))
    z = np.array(z)
    assert abs(z.mean()) < 4 / math.sqrt(len(z)) and 0.7 < z.std() < 1.3


def test_luminosity_distance_matches_paper_values():
    rows = [l.split()[:3] for l in open(os.path.join(GOLDEN, "distances_gpc.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) == 5
    for z, dl, tol in rows:
        assert abs(inputs.luminosity_distance_gpc(float(z)) / float(dl) - 1) < float(tol)


def test_psd_positive_and_T_suppressed():
    f = np.geomspace(1e-5, 0.1, 2000)
    S = inputs.psd_aet(f)
    assert np.all(S > 0)
    assert np.array_equal(S[0], S[1])
    assert S[2, 0] / S[0, 0] < 1e-6 and S[2, 0] / S[0, 0] < S[2, 500] / S[0, 500]


def test_grid_sizes_of_the_workloads():
    assert inputs.short_grid().grid.n == 125410 and inputs.short_grid().grid.k0 == 420
    g2 = inputs.year_grid(1).grid
    assert g2.n == 3355108 and g2.k0 == 336
