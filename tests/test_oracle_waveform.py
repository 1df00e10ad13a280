"""Pins of the oracle's waveform stage: harmonic-mode amplitude/phase
(Sec. II, Eq. amp_and_phase), the time-frequency map t_lm(f) (Eq. t_f), the
coalescence-time convention (t_coal at the maximum of f^2 A_22) and the
per-mode cut t_lm < 0.

The surrogate's physics against PhenomHM is "parity unpinned"; these tests pin
what the paper and mathematics fix: derivative consistency, the alignment
convention, the post-Newtonian low-frequency limit, 1/D_L scaling, mode
symmetries, and the band cuts by brute force."""
import math

import numpy as np
import pytest

from paper_2005_01827_amd import inputs

T0 = 3.15576e7
MODES = inputs.MODES_ALL


def _theta(M=3e6, q=0.3, a1=0.3, a2=-0.2, D=26.0, tref=50.25):
    return np.array([M, q, a1, a2, D, 2.14, 1.05, 2 * math.pi - 0.024, 0.62, 2.03, tref])


SOURCES = [
    _theta(),
    _theta(M=1e5, q=0.9, a1=0.95, a2=0.9),
    _theta(M=1e8, q=0.1, a1=-0.99, a2=0.99),
    _theta(M=2e6, q=1.0, a1=0.0, a2=0.0),
    _theta(M=4e7, q=0.05, a1=0.99, a2=-0.99),
]


@pytest.mark.parametrize("th", SOURCES)
@pytest.mark.parametrize("lm", MODES)
def test_time_is_minus_phase_derivative(oracle, th, lm):
    """t_lm(f) = t_coal - (1/2pi) dphi/df against a central finite difference of phi."""
    src = oracle.source(th, T0)
    M = src["M"]
    l, m = lm
    f = np.geomspace(1e-4 / M, 0.9 * 0.1 * m / M, 40)
    A, phi, dphi, t = oracle.mode(th, T0, l, m, f)
    h = f * 1e-5
    _, pp, _, _ = oracle.mode(th, T0, l, m, f + h)
    _, pm, _, _ = oracle.mode(th, T0, l, m, f - h)
    fd = (pp - pm) / (2 * h)
    # away from the join the phase is smooth; the FD truncation error is O(h^2 phi''')
    assert np.allclose(dphi, fd, rtol=2e-6, atol=1e-9 * np.abs(dphi).max())
    assert np.allclose(t, src["tcoal"] - dphi / (2 * math.pi), rtol=0, atol=1e-6 * src["tcoal"])


@pytest.mark.parametrize("th", SOURCES)
def test_second_derivative_and_c2_join(oracle, th):
    src = oracle.source(th, T0)
    fJ = src["fJ"]
    f = np.geomspace(0.2 * fJ, 5 * fJ, 31)
    h = f * 1e-5
    for which in (0, 1, 2):
        v = oracle.phase22_pieces(th, T0, which, f)
        vp = oracle.phase22_pieces(th, T0, which, f + h)
        vm = oracle.phase22_pieces(th, T0, which, f - h)
        fd1 = (vp[:, 0] - vm[:, 0]) / (2 * h)
        fd2 = (vp[:, 1] - vm[:, 1]) / (2 * h)
        ok = np.abs(f - fJ) > 2 * h if which == 2 else np.ones_like(f, bool)
        assert np.allclose(v[ok, 1], fd1[ok], rtol=1e-6)
        assert np.allclose(v[ok, 2], fd2[ok], rtol=1e-5)
    a = oracle.phase22_pieces(th, T0, 0, np.array([fJ]))[0]
    b = oracle.phase22_pieces(th, T0, 1, np.array([fJ]))[0]
    assert np.allclose(a, b, rtol=1e-10)
    # monotone time: second derivative negative on both sides
    assert a[2] < 0 and oracle.phase22_pieces(th, T0, 1, np.array([3 * fJ]))[0][2] < 0


@pytest.mark.parametrize("th", SOURCES)
def test_tcoal_at_peak_of_f2A22(oracle, th):
    src = oracle.source(th, T0)
    fp = src["fpeak"]
    _, _, _, t = oracle.mode(th, T0, 2, 2, np.array([fp]))
    assert abs(t[0] - src["tcoal"]) < 1e-6
    # brute force: f^2 A_22 on a fine grid peaks at fp
    f = np.linspace(0.5 * fp, 1.5 * fp, 200001)
    A, g = oracle.amp22(th, T0, f)
    fmax = f[np.argmax(f * f * A)]
    assert abs(fmax - fp) < 2 * (f[1] - f[0])
    # the derivative used by the bisection is the derivative of ln(f^2 A)
    fq = np.array([0.7 * fp, 0.9 * fp, 1.1 * fp])
    h = fq * 1e-6
    Ap, _ = oracle.amp22(th, T0, fq + h)
    Am, _ = oracle.amp22(th, T0, fq - h)
    _, gq = oracle.amp22(th, T0, fq)
    fd = (np.log((fq + h) ** 2 * Ap) - np.log((fq - h) ** 2 * Am)) / (2 * h)
    assert np.allclose(gq, fd, rtol=1e-6)


@pytest.mark.parametrize("th", SOURCES[:3] + SOURCES[4:])
def test_low_frequency_chirp_time(oracle, th):
    """Time to coalescence against the textbook post-Newtonian chirp time
    tau = 5M/(256 eta v^8) [1 + (4/3)(743/336 + 11 eta/4) v^2 - (8/5)(4 pi - beta) v^3]."""
    src = oracle.source(th, T0)
    M, eta = src["M"], src["eta"]
    q, a1, a2 = th[1], th[2], th[3]
    m1, m2 = 1 / (1 + q), q / (1 + q)
    beta = sum((113 / 12 * mi * mi + 25 / 4 * eta) * ai for mi, ai in ((m1, a1), (m2, a2)))
    Mf = np.geomspace(1e-6, 2e-5, 8)
    f = Mf / M
    _, _, _, t = oracle.mode(th, T0, 2, 2, f)
    tau = src["tcoal"] - t
    v = (math.pi * Mf) ** (1 / 3)
    pn = 5 * M / (256 * eta * v ** 8) * (1 + 4 / 3 * (743 / 336 + 11 * eta / 4) * v ** 2
                                          - 8 / 5 * (4 * math.pi - beta) * v ** 3)
    # the remainder is O(v^4) relative (plus the f_peak alignment shift, O(M))
    rel = np.abs(tau / pn - 1)
    assert np.all(rel < 60 * v ** 4 + 1e4 * M / pn)


def test_amplitude_scales_as_inverse_distance(oracle):
    th = _theta()
    f = np.geomspace(1e-5, 1e-2, 50)
    th2 = th.copy()
    th2[4] *= 3.7
    for l, m in MODES:
        A1, p1, _, _ = oracle.mode(th, T0, l, m, f)
        A2, p2, _, _ = oracle.mode(th2, T0, l, m, f)
        assert np.allclose(A1 / A2, 3.7, rtol=1e-13)
        assert np.array_equal(p1, p2)


def test_odd_m_modes_vanish_for_equal_masses(oracle):
    th = _theta(q=1.0, a1=0.4, a2=0.4)
    f = np.geomspace(1e-5, 1e-2, 20)
    for l, m in MODES:
        A, _, _, _ = oracle.mode(th, T0, l, m, f)
        if m % 2:
            assert np.all(A == 0.0)
        else:
            assert np.all(A > 0.0)


def test_face_on_inspiral_amplitude_is_newtonian_spa(oracle):
    """Face-on, low frequency: |h_+| of the (2,2) pair equals the leading-order
    stationary-phase amplitude sqrt(5/24) pi^(-2/3) Mc^(5/6) f^(-7/6) / D_L,
    once the Lorentzian bump and the logistic cut-off factors are divided out."""
    th = _theta(M=1e6, q=0.5)
    src = oracle.source(th, T0)
    M, eta, D = src["M"], src["eta"], src["Dl"]
    f = np.geomspace(1e-6, 1e-4, 5) / M * 1e2
    A, _ = oracle.amp22(th, T0, f)
    u = (f - src["fRD"]) / src["fd"]
    shape = (1 + 2.0 / (1 + u * u)) / (1 + np.exp(u))
    kp, kc = oracle.mode_weights(2, 2, 0.0, 0.0)
    hplus = abs(kp) * A / shape
    mc = eta ** 0.6 * M
    spa = math.sqrt(5 / 24) * math.pi ** (-2 / 3) * mc ** (5 / 6) * f ** (-7 / 6) / D
    assert np.allclose(hplus, spa, rtol=1e-12)


@pytest.mark.parametrize("lm", MODES)
def test_band_cut_brute_force(oracle, lm):
    """Bin k belongs to mode lm iff t_lm(k df) >= 0 and k df <= (m/2) 0.2 / M."""
    th = _theta(M=4e5, q=0.5, tref=3e4)
    T = 2.0 ** 21
    grid = inputs.Grid.from_band(T, 2e-4, 3e-2)
    t0 = 0.5 * T
    sp = oracle.sparse(th, grid, [lm], 16, t0)
    active, klo, khi, _ = sp["band"][0]
    k = grid.k0 + np.arange(grid.n)
    f = k * grid.df
    _, _, _, t = oracle.mode(th, t0, lm[0], lm[1], f)
    src = oracle.source(th, t0)
    fe = min(0.5 * lm[1] * 0.2 / src["M"], f[-1])
    member = (t >= 0) & (f <= fe)
    assert active == 1
    idx = np.nonzero(member)[0]
    assert k[idx[0]] == klo and k[idx[-1]] == khi
    assert np.all(member[idx[0]:idx[-1] + 1])
    # the root itself
    fs = sp["fband"][0][0]
    _, _, _, ts = oracle.mode(th, t0, lm[0], lm[1], np.array([fs, fs * (1 - 1e-15)]))
    assert ts[0] >= 0 and ts[1] < 1e-6


def test_mode_absent_when_it_ends_before_the_data(oracle):
    # a very heavy source whose ringdown cut lies below the band: no active mode
    th = _theta(M=1e9, q=0.5)
    grid = inputs.Grid.from_band(2.0 ** 20, 2e-3, 2e-2)
    sp = oracle.sparse(th, grid, MODES, 16, 0.5 * 2.0 ** 20)
    assert np.all(sp["band"][:, 0] == 0)


def test_invalid_parameters_rejected(oracle):
    for bad in (dict(q=1.2), dict(a1=1.0), dict(D=-1.0), dict(M=float("nan"))):
        with pytest.raises(ValueError):
            oracle.source(_theta(**bad), T0)


def test_higher_mode_stationary_phase_factor(oracle):
    """A harmonic m of the same orbital motion, h_m(t) = a(t) exp(-i m Phi(t)),
    has a stationary-phase amplitude sqrt(2/m) times that of m = 2 at the
    mapped frequency 2f/m.  Checked numerically on a synthetic chirp by FFT,
    then the oracle's A_lm(f) / A_22(2f/m) is checked to carry that factor
    times the leading-order amplitude ratio |H_lm/H_22| of its mode table."""
    n = 2 ** 18
    t = np.arange(n, dtype=float)
    forb = 0.004 + 0.05 * (t / n) ** 2           # orbital frequency, cycles/sample
    Phi = 2 * math.pi * np.cumsum(forb)
    edge = np.clip(np.minimum(t, n - 1 - t) / 4000.0, 0, 1)
    a = np.sin(0.5 * math.pi * edge) ** 2
    spec = {m: np.abs(np.fft.fft(a * np.exp(-1j * m * Phi))) for m in (2, 3, 4)}
    freqs = np.fft.fftfreq(n)
    # negative-frequency content of exp(-i m Phi) sits at -m forb
    def amp_at(m, f):
        k = np.argmin(np.abs(freqs + f))
        return spec[m][k - 40:k + 41].mean()
    for m in (3, 4):
        for f in (0.03, 0.05, 0.08):
            assert abs(amp_at(m, f) / amp_at(2, 2 * f / m) - math.sqrt(2 / m)) < 0.02

    th = _theta(M=3e6, q=0.3)
    src = oracle.source(th, T0)
    M, eta, dl = src["M"], src["eta"], src["delta"]
    ratios = {  # |H_lm / H_22| at leading order, as tabulated in the surrogate
        (3, 3): lambda v: 0.75 * math.sqrt(15 / 14) * dl * v,
        (4, 4): lambda v: 8 / 9 * math.sqrt(5 / 7) * (1 - 3 * eta) * v ** 2,
        (2, 1): lambda v: math.sqrt(2) / 3 * dl * v,
        (3, 2): lambda v: 1 / 3 * math.sqrt(5 / 7) * (1 - 3 * eta) * v ** 2,
        (4, 3): lambda v: 9 / (4 * math.sqrt(70)) * dl * (1 - 2 * eta) * v ** 3,
    }
    f = np.geomspace(1e-5, 5e-3, 7)
    for (l, m), R in ratios.items():
        A, _, _, _ = oracle.mode(th, T0, l, m, f)
        A22, _, _, _ = oracle.mode(th, T0, 2, 2, 2 * f / m)
        v = (math.pi * M * 2 * f / m) ** (1 / 3)
        assert np.allclose(A / A22, math.sqrt(2 / m) * np.array([R(x) for x in v]), rtol=1e-12)
