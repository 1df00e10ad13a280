"""Pins of the oracle's response stage (Sec. II, Eq. response and the TDI
combinations A = (Z-X)/sqrt2, E = (X-2Y+Z)/sqrt6, T = (X+Y+Z)/sqrt3).

The link transfer and the TDI combination are checked against a direct
evaluation of their time-domain definitions (two-time difference of the
metric perturbation along each arm; explicitly delayed first-generation
Michelson combination) for a complex monochromatic wave; the spin-weighted
harmonics against closed forms and orthonormality."""
import math

import numpy as np
import pytest

C = 299792458.0
L = 2.5e9 / C
AU = 1.495978707e11 / C
YEAR = 3.15576e7


def test_constellation_is_rigid_equilateral_tilted_60(oracle):
    for t in np.linspace(0.0, YEAR, 13):
        p = oracle.lisa_positions(t)
        for i in range(3):
            for j in range(i + 1, 3):
                assert abs(np.linalg.norm(p[i] - p[j]) - L) < 1e-12 * L
        c = p.mean(axis=0)
        al = 2 * math.pi * t / YEAR
        assert np.allclose(c, [AU * math.cos(al), AU * math.sin(al), 0.0], atol=1e-9 * AU)
        nrm = np.cross(p[1] - p[0], p[2] - p[0])
        cosang = abs(nrm[2]) / np.linalg.norm(nrm)
        assert abs(cosang - 0.5) < 1e-12
    assert np.allclose(oracle.lisa_positions(0.0), oracle.lisa_positions(YEAR), atol=1e-9 * AU)


def _basis(lam, beta, psi):
    k = -np.array([math.cos(beta) * math.cos(lam), math.cos(beta) * math.sin(lam), math.sin(beta)])
    u = np.array([math.sin(lam), -math.cos(lam), 0.0])
    v = np.array([-math.sin(beta) * math.cos(lam), -math.sin(beta) * math.sin(lam), math.cos(beta)])
    p = math.cos(psi) * u + math.sin(psi) * v
    q = -math.sin(psi) * u + math.cos(psi) * v
    ep = np.outer(p, p) - np.outer(q, q)
    ec = np.outer(p, q) + np.outer(q, p)
    return k, ep, ec


def _link_time_domain(f, tobs, pos, k, e, r, s):
    """Response of link s->r to h_ij(t, x) = e_ij exp(2 pi i f (t - k.x)),
    y(t) = [H(t - L - k.p_s) - H(t - k.p_r)] / (2 (1 - k.n)), at time tobs,
    divided by the wave at the constellation centre."""
    n = (pos[r] - pos[s]) / np.linalg.norm(pos[r] - pos[s])
    nen = n @ e @ n
    p0 = pos.mean(axis=0)
    # times are measured from tobs - k.p0 (the wave's phase at the centre),
    # which keeps the exponents small and the difference well conditioned
    H = lambda dt: nen * np.exp(2j * math.pi * f * dt)
    return (H(-L - k @ (pos[s] - p0)) - H(-k @ (pos[r] - p0))) / (2 * (1 - k @ n))


@pytest.mark.parametrize("f", [1e-5, 3e-3, 2e-2, 7e-2])
@pytest.mark.parametrize("cross", [0, 1])
def test_link_transfer_matches_time_domain_definition(oracle, f, cross):
    rng = np.random.default_rng(int(f * 1e6) + cross)
    for _ in range(4):
        lam, beta, psi = rng.uniform(0, 2 * math.pi), rng.uniform(-1.5, 1.5), rng.uniform(0, math.pi)
        t = rng.uniform(0, YEAR)
        pos = oracle.lisa_positions(t)
        k, ep, ec = _basis(lam, beta, psi)
        for r, s in ((0, 1), (1, 0), (0, 2), (2, 0), (1, 2), (2, 1)):
            ref = _link_time_domain(f, t, pos, k, ec if cross else ep, r, s)
            got = oracle.link(f, t, lam, beta, psi, r, s, cross)
            assert abs(got - ref) <= 1e-9 * max(abs(ref), 1e-300) + 1e-12 * math.pi * f * L


@pytest.mark.parametrize("f", [2e-5, 4e-3, 3e-2])
def test_tdi_matches_delayed_michelson_combination(oracle, f):
    """X(t) = y12(t) + y21(t-L) + y13(t-2L) + y31(t-3L) - y13(t) - y31(t-L)
    - y12(t-2L) - y21(t-3L), Y and Z by cyclic permutation (static
    constellation), for a wave with plus/cross weights kp, kc."""
    rng = np.random.default_rng(int(f * 1e7))
    lam, beta, psi = 1.3, -0.4, 0.7
    kp, kc = complex(0.3, -0.8), complex(-0.5, 0.25)
    t = 0.37 * YEAR
    pos = oracle.lisa_positions(t)
    k, ep, ec = _basis(lam, beta, psi)
    e = kp * ep + kc * ec

    def y(r, s, tau):
        # link s->r at time t - tau, relative to the centre wave at time t
        return _link_time_domain(f, t, pos, k, e, r, s) * np.exp(-2j * math.pi * f * tau)

    def mich(a, b, c):
        return (y(a, b, 0) + y(b, a, L) + y(a, c, 2 * L) + y(c, a, 3 * L)
                - y(a, c, 0) - y(c, a, L) - y(a, b, 2 * L) - y(b, a, 3 * L))

    X, Y, Z = mich(0, 1, 2), mich(1, 2, 0), mich(2, 0, 1)
    ref = np.array([(Z - X) / math.sqrt(2), (X - 2 * Y + Z) / math.sqrt(6), (X + Y + Z) / math.sqrt(3)])
    got, phorb = oracle.tdi(f, t, lam, beta, psi, kp, kc)
    scale = np.abs(ref).max()
    assert np.allclose(got, ref, rtol=0, atol=1e-9 * scale)
    assert abs(phorb - (-2 * math.pi * f * (k @ pos.mean(axis=0)))) < 1e-9 * (1 + abs(phorb))


def test_T_channel_suppressed_at_low_frequency(oracle):
    kp, kc = complex(1, 0), complex(0, 1)
    ratios = []
    for f in (1e-5, 1e-4, 1e-3):
        aet, _ = oracle.tdi(f, 0.2 * YEAR, 0.8, 0.3, 0.4, kp, kc)
        ratios.append(abs(aet[2]) / abs(aet[0]))
    # |T|/|A| ~ (2 pi f L)^2 at low frequency: two decades of f -> four of ratio
    assert ratios[0] < 1e-3 * ratios[2] * 10
    assert ratios[1] / ratios[0] > 50 and ratios[2] / ratios[1] > 50


CLOSED = {
    (2, 2): lambda th: math.sqrt(5 / (64 * math.pi)) * (1 + math.cos(th)) ** 2,
    (2, -2): lambda th: math.sqrt(5 / (64 * math.pi)) * (1 - math.cos(th)) ** 2,
    (2, 1): lambda th: math.sqrt(5 / (16 * math.pi)) * math.sin(th) * (1 + math.cos(th)),
    (2, -1): lambda th: math.sqrt(5 / (16 * math.pi)) * math.sin(th) * (1 - math.cos(th)),
    (2, 0): lambda th: math.sqrt(15 / (32 * math.pi)) * math.sin(th) ** 2,
    (3, 3): lambda th: -math.sqrt(21 / (2 * math.pi)) * math.cos(th / 2) ** 5 * math.sin(th / 2),
    (4, 4): lambda th: 3 * math.sqrt(7 / math.pi) * math.cos(th / 2) ** 6 * math.sin(th / 2) ** 2,
}


@pytest.mark.parametrize("lm", sorted(CLOSED))
def test_swsh_closed_forms(oracle, lm):
    l, m = lm
    for th in (0.0, 0.3, 1.05, 2.0, math.pi):
        for ph in (0.0, 0.9, 4.0):
            got = oracle.swsh(l, m, th, ph)
            ref = CLOSED[lm](th) * complex(math.cos(m * ph), math.sin(m * ph))
            assert abs(got - ref) < 1e-14


def test_swsh_orthonormal(oracle):
    xg, wg = np.polynomial.legendre.leggauss(40)
    th = np.arccos(xg)
    nph = 32
    ph = 2 * math.pi * np.arange(nph) / nph
    lms = [(l, m) for l in (2, 3, 4) for m in range(-l, l + 1)]
    Y = {lm: np.array([[oracle.swsh(lm[0], lm[1], t, p) for p in ph] for t in th]) for lm in lms}
    for a in lms:
        for b in lms:
            ip = np.sum(wg[:, None] * Y[a] * np.conj(Y[b])) * 2 * math.pi / nph
            assert abs(ip - (1.0 if a == b else 0.0)) < 1e-12


def test_mode_weights_polarization_states(oracle):
    # face-on (2,2): circular, h_x = -i h_+ ; edge-on: linear, h_x = 0
    kp, kc = oracle.mode_weights(2, 2, 0.0, 0.7)
    assert abs(kc + 1j * kp) < 1e-15 and abs(kp) > 0.1
    kp, kc = oracle.mode_weights(2, 2, math.pi / 2, 0.7)
    assert abs(kc) < 1e-15 and abs(kp) > 0.1
    # phi_ref enters as exp(-i m phi_ref)
    for l, m in ((2, 2), (3, 3), (2, 1), (4, 3)):
        a = oracle.mode_weights(l, m, 1.1, 0.0)
        b = oracle.mode_weights(l, m, 1.1, 0.4)
        rot = complex(math.cos(-m * 0.4), math.sin(-m * 0.4))
        assert abs(b[0] - a[0] * rot) < 1e-14 and abs(b[1] - a[1] * rot) < 1e-14
