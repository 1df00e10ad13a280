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
    mapped frequency 2f/m.  Checked numerically on a synthetic chirp by FFT
    (the mode table itself is pinned by the multipole tests below)."""
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


# ---------------------------------------------------------------------------
# The mode table against the radiation of a Newtonian circular binary.
#
# Far-zone field of a slow-motion source (Thorne 1980; G = c = 1, R = 1):
#   h_ab^TT = 4 sum_l (1/l!) [ N_{L-2} d^l I_{abL-2}/dt^l
#                              - (2l/(l+1)) N_{cL-2} eps_{cd(a} d^l J_{b)dL-2}/dt^l ]^TT
# with mass moments I_L = sum_A m_A y_A^L and current moments
# J_L = sum_A m_A Sym[y_A^{L-1} (y_A x v_A)].  Trace terms of the moments only
# feed lower l, so the l-th multipole projected onto _{-2}Y_lm needs no trace
# removal.  Time derivatives are spectral (one orbit, exact for the harmonic
# content), and h_lm = int (h_+ - i h_x) conj(_{-2}Y_lm) dOmega by
# Gauss-Legendre x uniform quadrature.  Nothing here restates the oracle's
# table: the coefficients come out of the point-mass sums.
# ---------------------------------------------------------------------------
_EPS = np.zeros((3, 3, 3))
for _a, _b, _c in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
    _EPS[_a, _b, _c], _EPS[_a, _c, _b] = 1.0, -1.0


def _multipole_modes(oracle, q, r=400.0, nt=32, nth=24, nph=48):
    """{(l,m): H_lm/H_22} of a circular binary of mass ratio q at separation
    r (total mass 1), the e^{-i m Phi} orbital dependence removed; v = r^-1/2."""
    m1, m2 = 1 / (1 + q), q / (1 + q)
    om = r ** -1.5
    ph = np.arange(nt) * 2 * math.pi / nt
    n = np.stack([np.cos(ph), np.sin(ph), 0 * ph], -1)
    lam = np.stack([-np.sin(ph), np.cos(ph), 0 * ph], -1)
    bodies = [(m1, m2 * r * n, m2 * r * om * lam), (m2, -m1 * r * n, -m1 * r * om * lam)]
    x, w = np.polynomial.legendre.leggauss(nth)
    th = np.arccos(x)
    phs = np.arange(nph) * 2 * math.pi / nph
    TH, PH = np.meshgrid(th, phs, indexing="ij")
    N = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], -1)
    eth = np.stack([np.cos(TH) * np.cos(PH), np.cos(TH) * np.sin(PH), -np.sin(TH)], -1)
    eph = np.stack([-np.sin(PH), np.cos(PH), 0 * PH], -1)
    k = np.fft.fftfreq(nt, d=1.0 / nt)

    def deriv(a, p):
        A = np.fft.fft(a, axis=0) * ((1j * om * k) ** p).reshape((-1,) + (1,) * (a.ndim - 1))
        return np.fft.ifft(A, axis=0).real

    def mass(l):
        s = sum(mA * np.einsum("ta,tb,txy->txyab", y, y, np.einsum("tc,xyc->txy", y, N) ** (l - 2))
                for mA, y, _ in bodies)
        return 4 / math.factorial(l) * deriv(s, l)

    def current(l):
        s = 0
        for mA, y, v in bodies:
            wv = np.cross(y, v)
            yN, wN = np.einsum("tc,xyc->txy", y, N), np.einsum("tc,xyc->txy", wv, N)
            S = (np.einsum("tb,td,txy->txybd", wv, y, yN ** (l - 2))
                 + np.einsum("tb,td,txy->txybd", y, wv, yN ** (l - 2)))
            if l > 2:
                S = S + (l - 2) * np.einsum("tb,td,txy->txybd", y, y, wN * yN ** (l - 3))
            s = s + mA * S / l
        c = np.einsum("cda,xyc,txybd->txyab", _EPS, N, deriv(s, l))
        return -(4 / math.factorial(l)) * (2 * l / (l + 1)) * 0.5 * (c + np.swapaxes(c, -1, -2))

    def project(h, l, m):
        hp = 0.5 * (np.einsum("txyab,xya,xyb->txy", h, eth, eth) - np.einsum("txyab,xya,xyb->txy", h, eph, eph))
        hc = 0.5 * (np.einsum("txyab,xya,xyb->txy", h, eth, eph) + np.einsum("txyab,xya,xyb->txy", h, eph, eth))
        Y = np.array([[oracle.swsh(l, m, a, b) for b in phs] for a in th])
        hlm = np.einsum("txy,xy,x->t", hp - 1j * hc, np.conj(Y), w) * (2 * math.pi / nph)
        return (hlm * np.exp(1j * m * ph)).mean()

    out = {(2, 2): project(mass(2), 2, 2), (3, 3): project(mass(3), 3, 3), (4, 4): project(mass(4), 4, 4),
           (2, 1): project(current(2), 2, 1), (3, 2): project(current(3), 3, 2), (4, 3): project(current(4), 4, 3)}
    return {lm: h / out[(2, 2)] for lm, h in out.items()}, om ** (1 / 3)


@pytest.mark.parametrize("q", [0.15, 0.5, 0.85])
def test_mode_amplitudes_from_multipole_radiation(oracle, q):
    """A_lm(f) / (sqrt(2/m) A_22(2f/m)) equals |H_lm/H_22| of the multipole
    radiation at the same orbital velocity: this pins the delta, (1 - 3 eta)
    and delta (1 - 2 eta) dependence and every numeric prefactor."""
    H, v = _multipole_modes(oracle, q)
    th = _theta(M=3e6, q=q)
    M = oracle.source(th, T0)["M"]
    for (l, m), h in H.items():
        f = m * v ** 3 / (2 * math.pi * M)          # (pi M 2f/m)^(1/3) = v
        A, _, _, _ = oracle.mode(th, T0, l, m, np.array([f]))
        A22, _, _, _ = oracle.mode(th, T0, 2, 2, np.array([2 * f / m]))
        assert abs(A[0] / (math.sqrt(2 / m) * A22[0]) / abs(h) - 1) < 1e-10, ((l, m), q)


def test_mode_phase_constants_by_stationary_phase(oracle):
    """The constant phase of every mode relative to the (2,2) mode.

    A synthetic chirp carries the time-domain modes h_lm = a(t) H_lm
    e^{-i m Phi(t)} with the multipole coefficients H_lm, their partners
    h_{l,-m} = (-1)^l conj(h_lm), and the harmonics _{-2}Y_lm of a fixed
    direction.  Its h_+ and h_x are Fourier transformed (e^{-2 pi i f t}, as
    the likelihood uses); dividing by the oracle's plus and cross weights of
    each pair leaves that mode's frequency-domain function Z_lm.  At one
    orbital frequency F (mode frequency mF) the combinations
      arg Z_lm(mF) - (m/2) arg Z_22(2F)      (even m: 44, 32),
      arg Z_lm(mF) - (m/2) arg Z_22(2F)  mod pi   (odd m: the (2,2)
          alignment fixes the orbital phase only up to pi, which for odd m is
          the relabelling phi_ref -> phi_ref + pi),
      arg Z_lm(3F) - 3 arg Z_21(F)           (33 and 43 against 21)
    do not depend on F, and must equal the oracle's phi_lm - (m/2) phi_22 and
    phi_lm - 3 phi_21 at matching frequencies."""
    q = 0.4
    H, _ = _multipole_modes(oracle, q)
    th = _theta(M=3e6, q=q)
    n = 2 ** 18
    t = np.arange(n, dtype=float)
    forb = 0.004 + 0.02 * (t / n) ** 2                       # orbital frequency [cycles/sample]
    Phi = 2 * math.pi * np.cumsum(forb)
    edge = np.clip(np.minimum(t, n - 1 - t) / 4000.0, 0, 1)
    a = np.sin(0.5 * math.pi * edge) ** 2
    iota, phr = 0.7, 0.4

    def Z(l, m, f):
        """plus- and cross-derived frequency-domain function of mode (l,m) at f"""
        hlm = a * H[(l, m)] * np.exp(-1j * m * Phi)
        s = hlm * oracle.swsh(l, m, iota, phr) + (-1) ** l * np.conj(hlm) * oracle.swsh(l, -m, iota, phr)
        e = np.exp(-2j * math.pi * f * t)
        kp, kc = oracle.mode_weights(l, m, iota, phr)
        return np.sum(s.real * e) / kp, np.sum(-s.imag * e) / kc

    M = oracle.source(th, T0)["M"]
    fo = np.array([1e-4 / M * 1e-2, 3e-4 / M * 1e-2])          # orbital frequencies for the oracle [Hz]

    def oracle_phase(l, m, F):
        return oracle.mode(th, T0, l, m, m * F)[1]

    def wrap(x, per=2 * math.pi):
        return (x + per / 2) % per - per / 2

    for F in (0.006, 0.01):                                  # orbital frequency of the chirp
        z22 = Z(2, 2, 2 * F)
        z21 = Z(2, 1, F)
        for (l, m) in MODES[1:]:
            zlm = Z(l, m, m * F)
            want = oracle_phase(l, m, fo) - m / 2 * oracle_phase(2, 2, fo)
            per = 2 * math.pi if m % 2 == 0 else math.pi
            for k in (0, 1):                                 # plus, cross
                meas = np.angle(zlm[k]) - m / 2 * np.angle(z22[k])
                assert np.all(np.abs(wrap(want - meas, per)) < 3e-3), ((l, m), F, k, want, meas)
                assert abs(abs(zlm[k]) / abs(z22[k]) / (math.sqrt(2 / m) * abs(H[(l, m)])) - 1) < 1e-3
            if m == 3:
                want3 = oracle_phase(l, m, fo) - 3 * oracle_phase(2, 1, fo)
                for k in (0, 1):
                    meas3 = np.angle(zlm[k]) - 3 * np.angle(z21[k])
                    assert np.all(np.abs(wrap(want3 - meas3)) < 3e-3), ((l, m), F, k, want3, meas3)


def _tf2_time_from_energy_flux(eta, M, v):
    """Time to coalescence (up to a constant) of the point-mass TaylorF2
    approximant: dt/dv = -M (dE/dv)/F with the binding energy E to 3PN and the
    flux F to 3.5PN, the ratio re-expanded in v to relative order v^7 and
    integrated term by term (the construction TaylorF2's phase comes from)."""
    pi, g = math.pi, 0.5772156649015329
    e = [1, -0.75 - eta / 12, -27 / 8 + 19 * eta / 8 - eta ** 2 / 24,
         -675 / 64 + (34445 / 576 - 205 * pi ** 2 / 96) * eta - 155 * eta ** 2 / 96 - 35 * eta ** 3 / 5184]
    f = [1, 0, -1247 / 336 - 35 * eta / 12, 4 * pi, -44711 / 9072 + 9271 * eta / 504 + 65 * eta ** 2 / 18,
         (-8191 / 672 - 583 * eta / 24) * pi,
         6643739519 / 69854400 + 16 * pi ** 2 / 3 - 1712 * g / 105 - 856 / 105 * math.log(16)
         + (-134543 / 7776 + 41 * pi ** 2 / 48) * eta - 94403 * eta ** 2 / 3024 - 775 * eta ** 3 / 324,
         (-16285 / 504 + 214745 * eta / 1728 + 193385 * eta ** 2 / 3024) * pi]
    f6_log = -2 * 856 / 105                    # coefficient of ln v in f_6 (ln 16x = ln 16 + 2 ln v)
    # E = -(eta/2) v^2 sum e_k v^2k  ->  -dE/dv = eta v sum (k+1) e_k v^2k;  F = 32/5 eta^2 v^10 sum f_k v^k
    num = np.zeros(8)
    for k, ek in enumerate(e):
        num[2 * k] = (k + 1) * ek
    quo = np.zeros(8)
    for k in range(8):
        quo[k] = num[k] - sum(f[j] * quo[k - j] for j in range(1, k + 1))
    tot = sum(quo[k] * v ** (k - 8) / (k - 8) for k in range(8))
    tot = tot - f6_log * (-np.log(v) / (2 * v * v) - 1 / (4 * v * v))   # int v^-3 ln v dv
    return 5 * M / (32 * eta) * tot


@pytest.mark.parametrize("q", [1.0, 0.3, 0.05])
def test_taylorf2_against_energy_and_flux(oracle, q):
    """The (2,2) inspiral time t(f) = t_coal - phi'(f)/2pi of the oracle, whose
    TaylorF2 coefficients p2..p7 enter it, against the point-mass energy-flux
    construction, to 1e-12 relative in time differences (a one-unit change in
    any rational coefficient of p4..p7 moves it by >= 1e-9)."""
    th = _theta(M=2e6, q=q, a1=0.0, a2=0.0)
    src = oracle.source(th, T0)
    M, eta = src["M"], src["eta"]
    Mf = np.array([2e-4, 1e-3, 4e-3, 7e-3])
    _, _, _, t = oracle.mode(th, T0, 2, 2, Mf / M)
    tp = _tf2_time_from_energy_flux(eta, M, (math.pi * Mf) ** (1 / 3))
    d_or, d_pn = t[1:] - t[0], tp[1:] - tp[0]
    assert np.all(np.abs(d_or / d_pn - 1) < 1e-12), (d_or / d_pn - 1)


def test_remnant_fits_against_reference_values(oracle):
    """Final spin, radiated energy and the (2,2,0) ringdown against values the
    fits are meant to reproduce: numerical relativity for an equal-mass
    non-spinning merger (a_f = 0.6865, E_rad = 0.0484 M; Scheel et al. 2009),
    the test-mass limits (a_f -> spin of the large body; E_rad/eta -> 1 -
    sqrt(8/9), the ISCO binding energy), and Kerr quasi-normal frequencies
    M omega = 0.3737 - 0.0890 i (a = 0) and 0.6716 - 0.0649 i (a = 0.9)
    (Leaver 1985; Berti, Cardoso & Will 2006), to the fit's few-percent."""
    s = oracle.source(_theta(q=1.0, a1=0.0, a2=0.0), T0)
    assert abs(s["af"] - 0.6865) < 2e-3
    assert abs(1 - s["Mfin"] / s["M"] - 0.0484) < 1e-3
    s = oracle.source(_theta(q=1e-4, a1=0.37, a2=-0.5), T0)
    assert abs(s["af"] - 0.37) < 2e-3
    assert abs((1 - s["Mfin"] / s["M"]) / s["eta"] / (1 - math.sqrt(8 / 9)) - 1) < 0.03
    # choose a1 so that the final spin is exactly the target (a_f is linear in a1)
    q = 0.2
    base = oracle.source(_theta(q=q, a1=0.0, a2=0.0), T0)["af"]
    x1 = 1 / (1 + q)
    for af, w_ref, wi_ref in ((0.0, 0.3737, 0.0890), (0.9, 0.6716, 0.0649)):
        s = oracle.source(_theta(q=q, a1=(af - base) / x1 ** 2, a2=0.0), T0)
        assert abs(s["af"] - af) < 1e-12
        w = 2 * math.pi * s["fRD"] * s["Mfin"]
        wi = 2 * math.pi * s["fd"] * s["Mfin"]
        assert abs(w / w_ref - 1) < 0.02 and abs(wi / wi_ref - 1) < 0.04, (af, w, wi)
