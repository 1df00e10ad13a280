"""LISA-frame coordinates and the eight sky modes (Sec. II, sampling in the
LISA frame; Sec. III.B, walkers started at the eight sky modes).

The frame module is product host code written from the constellation reading;
these pins check it against what the geometry fixes: the oracle's own
spacecraft positions (an independent implementation of the same
constellation), closed-form arrival times, round trips, and the symmetries of
the oracle's response that make the eight modes degenerate."""
import math

import numpy as np
import pytest

from paper_2005_01827_amd import inputs
from paper_2005_01827_amd import lisaframe as LF

T0 = inputs.YEAR_S
TIMES = np.array([0.0, 1.234e6, 0.25 * T0, 0.5 * T0, 0.9 * T0, T0 + 50.25, 2.7e7])


def test_frame_axes_follow_the_oracle_constellation(oracle):
    """z_L is normal to the oracle's spacecraft triangle, x_L points from its
    centroid to spacecraft 0, and the axes are right-handed and orthonormal."""
    for t in TIMES:
        pos = oracle.lisa_positions(t)                 # [3][3] light-seconds
        ax, p0 = LF.frame_axes(t)
        c = pos.mean(axis=0)
        assert np.allclose(p0, c, rtol=0, atol=1e-9)
        for i, j in ((0, 1), (1, 2), (2, 0)):
            arm = pos[j] - pos[i]
            assert abs(np.dot(arm, ax[2])) < 1e-12 * np.linalg.norm(arm)
        x = (pos[0] - c) / np.linalg.norm(pos[0] - c)
        assert np.allclose(ax[0], x, rtol=0, atol=1e-12)
        assert np.allclose(ax @ ax.T, np.eye(3), rtol=0, atol=1e-14)
        assert np.allclose(np.cross(ax[0], ax[1]), ax[2], rtol=0, atol=1e-14)
        # the plane is tilted by 60 degrees to the ecliptic
        assert abs(abs(ax[2][2]) - 0.5) < 1e-12


def test_arrival_time_closed_forms():
    """A source at the ecliptic pole: the centre stays in the ecliptic plane,
    so t_L = t_SSB.  A source in the direction of the constellation centre:
    the wave reaches LISA one AU of light travel before the barycentre."""
    R = LF.AU_M / LF.C_SI
    for t in TIMES:
        tL, _, _, _ = LF.ssb_to_lisa(t, 0.3, 0.5 * math.pi, 1.0)
        assert abs(tL - t) < 1e-8
        # centre direction at the arrival time: iterate the closed form
        al = 2.0 * math.pi * (t - R) / inputs.YEAR_S
        tL, lamL, betaL, _ = LF.ssb_to_lisa(t, al % (2 * math.pi), 0.0, 1.0)
        assert abs(tL - (t - R)) < 1e-6


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_round_trips(seed):
    rng = np.random.default_rng(seed)
    n = 500
    t = rng.uniform(0, 3 * inputs.YEAR_S, n)
    lam = rng.uniform(0, 2 * math.pi, n)
    beta = np.arcsin(rng.uniform(-0.999, 0.999, n))
    psi = rng.uniform(0, math.pi, n)
    tL, lamL, betaL, psiL = LF.ssb_to_lisa(t, lam, beta, psi)
    t2, lam2, beta2, psi2 = LF.lisa_to_ssb(tL, lamL, betaL, psiL)
    wrap = lambda d, p: np.abs(np.mod(d + 0.5 * p, p) - 0.5 * p)
    assert np.max(np.abs(t2 - t)) < 1e-7
    assert np.max(wrap(lam2 - lam, 2 * math.pi)) < 1e-12
    assert np.max(np.abs(beta2 - beta)) < 1e-12
    assert np.max(wrap(psi2 - psi, math.pi)) < 1e-11
    # and the other way round, from LISA-frame values
    tL3, lamL3, betaL3, psiL3 = LF.ssb_to_lisa(*LF.lisa_to_ssb(tL, lamL, betaL, psiL))
    assert np.max(np.abs(tL3 - tL)) < 1e-7
    assert np.max(wrap(lamL3 - lamL, 2 * math.pi)) < 1e-12
    assert np.max(wrap(psiL3 - psiL, math.pi)) < 1e-11
    # the arrival-time offset is at most one AU of light travel
    assert np.max(np.abs(tL - t)) <= LF.AU_M / LF.C_SI * (1 + 1e-9)


def test_physical_parameter_round_trip():
    th = inputs.year_grid(64).walkers
    thL = LF.physical_to_lisa(th, T0)
    back = LF.lisa_to_physical(thL, T0)
    assert np.allclose(back[:, [0, 1, 2, 3, 4, 5, 6, 8]], th[:, [0, 1, 2, 3, 4, 5, 6, 8]], rtol=1e-13, atol=1e-12)
    assert np.allclose(back[:, 10], th[:, 10], rtol=0, atol=1e-7)
    x = LF.to_sampling_lisa(thL)
    assert np.allclose(LF.from_sampling_lisa(x), thL, rtol=1e-13, atol=1e-13)


def _tdi_ssb(oracle, f, t, thL_sky, kp, kc):
    """The oracle's A, E, T transfer for a unit plus (kp) / cross (kc) wave
    whose LISA-frame angles at time t are thL_sky = (lambda_L, beta_L,
    psi_L); positions are held at time t."""
    lamL, betaL, psiL = thL_sky
    _, lam, beta, psi = LF.lisa_to_ssb(t, lamL, betaL, psiL)
    aet, _ = oracle.tdi(f, t, float(lam), float(beta), float(psi), kp, kc)
    return aet


@pytest.mark.parametrize("f", [1e-4, 3e-3, 2e-2])
def test_reflection_mode_is_exact(oracle, f):
    """beta_L -> -beta_L with psi_L -> pi - psi_L leaves the oracle's plus
    response unchanged and negates its cross response, at every frequency
    (all arms lie in the constellation plane)."""
    rng = np.random.default_rng(4)
    for _ in range(5):
        t = rng.uniform(0, inputs.YEAR_S)
        lamL, betaL, psiL = rng.uniform(0, 2 * math.pi), math.asin(rng.uniform(-0.95, 0.95)), rng.uniform(0, math.pi)
        for kp, kc, sgn in ((1.0, 0.0, 1.0), (0.0, 1.0, -1.0)):
            a = _tdi_ssb(oracle, f, t, (lamL, betaL, psiL), kp, kc)
            b = _tdi_ssb(oracle, f, t, (lamL, -betaL, math.pi - psiL), kp, kc)
            assert np.allclose(b, sgn * a, rtol=0, atol=1e-9 * np.abs(a).max()), (f, a, b)


def test_quarter_turn_modes_at_low_frequency(oracle):
    """lambda_L + k pi/2 with psi_L + k pi/2 gives the same A and E in the
    low-frequency limit (to O(f L / c)); at 20 mHz, where the arm transfer
    matters, it does not."""
    rng = np.random.default_rng(5)
    for _ in range(5):
        t = rng.uniform(0, inputs.YEAR_S)
        lamL, betaL, psiL = rng.uniform(0, 2 * math.pi), math.asin(rng.uniform(-0.9, 0.9)), rng.uniform(0, math.pi)
        for kp, kc in ((1.0, 0.0), (0.0, 1.0)):
            ref_lo = _tdi_ssb(oracle, 1e-5, t, (lamL, betaL, psiL), kp, kc)[:2]
            ref_hi = _tdi_ssb(oracle, 2e-2, t, (lamL, betaL, psiL), kp, kc)[:2]
            worst_hi = 0.0
            for k in (1, 2, 3):
                img = (lamL + k * 0.5 * math.pi, betaL, psiL + k * 0.5 * math.pi)
                lo = _tdi_ssb(oracle, 1e-5, t, img, kp, kc)[:2]
                hi = _tdi_ssb(oracle, 2e-2, t, img, kp, kc)[:2]
                scale = np.abs(ref_lo).max()
                assert np.max(np.abs(lo - ref_lo)) < 2e-3 * scale, (k, lo, ref_lo)
                worst_hi = max(worst_hi, np.max(np.abs(hi - ref_hi)) / np.abs(ref_hi).max())
            assert worst_hi > 0.05


def test_sky_modes_follow_the_paper():
    """Eight modes: longitudes the true one plus k pi/2, each above and below
    the constellation plane; the first is the input; the other parameters
    move only by the documented maps."""
    thL = LF.physical_to_lisa(inputs.year_grid(1).injection, T0)
    m = LF.sky_modes(thL)
    assert m.shape == (8, 11)
    assert np.array_equal(m[0], np.concatenate([thL[:9], [thL[9] % math.pi], thL[10:]]))
    lam = np.sort(np.mod(m[:4, 7] - thL[7], 2 * math.pi))
    assert np.allclose(lam, [0, 0.5 * math.pi, math.pi, 1.5 * math.pi], atol=1e-12)
    assert np.allclose(m[:4, 8], thL[8]) and np.allclose(m[4:, 8], -thL[8])
    assert np.allclose(m[4:, 7], m[:4, 7])
    assert np.allclose(m[4:, 6], math.pi - thL[6])
    for col in (0, 1, 2, 3, 4, 5, 10):
        assert np.all(m[:, col] == thL[col])
    x = LF.sky_mode_walkers(thL, 3, 4, 1e-6, 9)
    assert x.shape == (3, 32, 11)
    # 4 walkers per temperature at each mode, near it
    xm = LF.to_sampling_lisa(m)
    for j in range(8):
        blk = x[:, 4 * j:4 * (j + 1)]
        assert np.allclose(blk[..., 8], xm[j, 8], atol=1e-4)


def test_lisa_prior_carries_the_table_one_prior():
    """The LISA-frame prior is the SSB box prior of the converted point plus
    ln |J|; the map is close to volume-preserving (a rotation of the sky and
    of the polarisation angle, and a delay that changes slowly with time)."""
    thL = LF.physical_to_lisa(inputs.year_grid(32).walkers, T0)
    x = LF.to_sampling_lisa(thL)
    lj = LF.log_jacobian(x, T0)
    ln_tref = -np.log(LF.sampling_lisa_to_ssb(x, T0)[:, 10])    # d ln t_ref = dt / t_ref
    assert np.all(np.abs(lj - ln_tref) < 1e-3)
    lp = LF.lisa_logprior(T0)(x)
    assert np.all(np.isfinite(lp))
    assert np.allclose(lp, lj)
    bad = x.copy()
    bad[:, 9] = math.pi + 0.1
    assert np.all(np.isneginf(LF.lisa_logprior(T0)(bad)))


def test_sky_modes_inside_the_prior_when_the_merger_is_late_enough():
    """The prior is the SSB one carried over, and a sky mode moves the SSB
    arrival time by at most 2 AU/c (about 998 s): with t_ref = 2000 s every
    mode has a finite prior; with t_ref = 50.25 s (Binary 1) the modes whose
    SSB time falls below 1 s carry none."""
    au_s = LF.AU_M / LF.C_SI
    for tref, all_inside in ((2000.0, True), (50.25, False)):
        th = inputs.year_grid(1).injection.copy()
        th[10] = tref
        thL = LF.physical_to_lisa(th, T0)
        m = LF.sky_modes(thL)
        t_ssb = LF.lisa_to_physical(m, T0)[:, 10]
        assert np.all(np.abs(t_ssb - tref) <= 2.0 * au_s + 1.0)
        lp = LF.lisa_logprior(T0)(LF.to_sampling_lisa(m))
        assert np.isfinite(lp[0])
        assert np.array_equal(np.isfinite(lp), t_ssb >= 1.0)
        assert np.all(np.isfinite(lp)) == all_inside
