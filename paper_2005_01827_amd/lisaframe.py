"""LISA-frame sky and time coordinates, and the eight sky modes.

Sec. II (after the TDI combinations): the extrinsic parameters lambda, beta,
psi and t_ref enter the response in the solar-system-barycentre (SSB)
frame, but the sampler moves them in the LISA frame and converts them to the
SSB frame before each waveform.  Sec. III.B: in the LISA frame the sky
posterior generally has eight modes, at the true longitude plus multiples of
pi/2 and at the true latitude above or below the constellation plane, and
the sampler starts 4 walkers per temperature at each of them.

The paper takes the frame from Marsat et al. (2020), which it does not
reproduce.  Reading used here: the frame is attached to the constellation
model of the response (a rigid equilateral triangle of side L whose centre
moves on a circular 1-AU ecliptic orbit of period 1 yr, plane tilted by 60
degrees, orbital and cartwheel phases zero at t = 0), at the time t_L at
which the wave reaches the constellation centre:
  z_L  unit normal of the constellation plane, (s1 - s0) x (s2 - s0);
  x_L  from the centre towards spacecraft 0;  y_L = z_L x x_L;
  (lambda_L, beta_L)  the source direction in (x_L, y_L, z_L);
  psi_L  the polarisation angle built the same way as the SSB one (basis
         u = (sin l, -cos l, 0), v = (-sin b cos l, -sin b sin l, cos b) in
         the frame's own axes), for the same physical polarisation;
  t_L  = t_SSB + k.p0(t_L)/c, with k the propagation direction and p0 the
         constellation centre: the arrival time at LISA.
LISA -> SSB is explicit; SSB -> LISA solves the arrival-time equation by
fixed-point iteration (contraction about 1e-4 per step).

Why eight modes: every arm lies in the constellation plane, so a reflection
of the source through that plane (beta_L -> -beta_L) with psi_L -> pi - psi_L
and the cross polarisation negated (iota -> pi - iota for the (2,2) mode)
leaves every arm projection n.e.n and every k.n unchanged: the response is
the same at all frequencies for a constellation held still.  A rotation of
the source by pi/2 about z_L turns the in-plane, traceless low-frequency
response tensors of A and E into their negatives (they rotate by twice the
angle), and psi_L -> psi_L + pi/2 negates the polarisation tensor: together
they leave A and E unchanged in the low-frequency limit (arm transfer
factors -> 1), for every mode.  sky_modes() applies exactly these maps.

Host-side, numpy only: the conversion touches 4 of 11 numbers per walker.
"""
from __future__ import annotations

import math

import numpy as np

from . import inputs

AU_M = 1.495978707e11
YEAR_S = inputs.YEAR_S
C_SI = inputs.C_SI
LARM_M = inputs.LARM_M


def constellation(t):
    """Centre p0[..., 3] and spacecraft positions s[..., 3, 3] in
    light-seconds at SSB time t (any shape), from the model above."""
    t = np.asarray(t, dtype=np.float64)
    R = AU_M / C_SI
    ecc = LARM_M / (2.0 * math.sqrt(3.0) * AU_M)
    al = 2.0 * math.pi * t / YEAR_S
    p0 = np.stack([R * np.cos(al), R * np.sin(al), np.zeros_like(al)], axis=-1)
    sc = []
    for i in range(3):
        b = 2.0 * math.pi * i / 3.0
        off = np.stack([ecc * R * (0.5 * np.cos(2.0 * al - b) - 1.5 * math.cos(b)),
                        ecc * R * (0.5 * np.sin(2.0 * al - b) - 1.5 * math.sin(b)),
                        -ecc * R * math.sqrt(3.0) * np.cos(al - b)], axis=-1)
        sc.append(p0 + off)
    return p0, np.stack(sc, axis=-2)


def frame_axes(t):
    """LISA-frame axes (x_L, y_L, z_L) as SSB unit vectors [..., 3, 3] (rows)
    and the centre p0 [..., 3], at time t."""
    p0, s = constellation(t)
    z = np.cross(s[..., 1, :] - s[..., 0, :], s[..., 2, :] - s[..., 0, :])
    z /= np.linalg.norm(z, axis=-1, keepdims=True)
    x = s[..., 0, :] - p0
    x -= np.sum(x * z, axis=-1, keepdims=True) * z
    x /= np.linalg.norm(x, axis=-1, keepdims=True)
    y = np.cross(z, x)
    return np.stack([x, y, z], axis=-2), p0


def _direction(lam, beta):
    cb = np.cos(beta)
    return np.stack([cb * np.cos(lam), cb * np.sin(lam), np.sin(beta)], axis=-1)


def _pol_basis(lam, beta):
    u = np.stack([np.sin(lam), -np.cos(lam), np.zeros_like(lam)], axis=-1)
    v = np.stack([-np.sin(beta) * np.cos(lam), -np.sin(beta) * np.sin(lam), np.cos(beta)], axis=-1)
    return u, v


def _angles(n):
    beta = np.arcsin(np.clip(n[..., 2], -1.0, 1.0))
    lam = np.mod(np.arctan2(n[..., 1], n[..., 0]), 2.0 * math.pi)
    return lam, beta


def lisa_to_ssb(tL, lamL, betaL, psiL):
    """(t_L, lambda_L, beta_L, psi_L) -> (t_SSB, lambda, beta, psi); arrays
    broadcast.  lambda in [0, 2 pi), psi in [0, pi)."""
    tL, lamL, betaL, psiL = np.broadcast_arrays(*(np.asarray(a, dtype=np.float64) for a in (tL, lamL, betaL, psiL)))
    ax, p0 = frame_axes(tL)
    nL = _direction(lamL, betaL)
    n = np.einsum("...i,...ij->...j", nL, ax)            # SSB components
    uL, vL = _pol_basis(lamL, betaL)
    epL = np.cos(psiL)[..., None] * uL + np.sin(psiL)[..., None] * vL
    ep = np.einsum("...i,...ij->...j", epL, ax)
    lam, beta = _angles(n)
    u, v = _pol_basis(lam, beta)
    psi = np.mod(np.arctan2(np.sum(ep * v, -1), np.sum(ep * u, -1)), math.pi)
    k = -n
    t = tL - np.sum(k * p0, axis=-1)
    return t, lam, beta, psi


def ssb_to_lisa(t, lam, beta, psi, iters: int = 8):
    """(t_SSB, lambda, beta, psi) -> (t_L, lambda_L, beta_L, psi_L)."""
    t, lam, beta, psi = np.broadcast_arrays(*(np.asarray(a, dtype=np.float64) for a in (t, lam, beta, psi)))
    n = _direction(lam, beta)
    k = -n
    tL = t.copy()
    for _ in range(iters):
        p0, _ = constellation(tL)
        tL = t + np.sum(k * p0, axis=-1)
    ax, _ = frame_axes(tL)
    nL = np.einsum("...ij,...j->...i", ax, n)
    u, v = _pol_basis(lam, beta)
    ep = np.cos(psi)[..., None] * u + np.sin(psi)[..., None] * v
    epL = np.einsum("...ij,...j->...i", ax, ep)
    lamL, betaL = _angles(nL)
    uL, vL = _pol_basis(lamL, betaL)
    psiL = np.mod(np.arctan2(np.sum(epL * vL, -1), np.sum(epL * uL, -1)), math.pi)
    return tL, lamL, betaL, psiL


# ---------------------------------------------------------------------------
# Parameters and sampling coordinates
# ---------------------------------------------------------------------------
# Physical parameters with LISA-frame extrinsics:
#   (M_T, q, a1, a2, D_L, phi_ref, iota, lambda_L, beta_L, psi_L, tau_L)
# where tau_L = t_L - t0 [s] (the arrival time at LISA relative to t0; it may
# be negative, so it is sampled linearly).  Sampling coordinates:
#   (ln M_T, q, a1, a2, ln D_L, phi_ref, cos iota, lambda_L, sin beta_L, psi_L, tau_L).

def physical_to_lisa(th, t0):
    """SSB physical parameters [..., 11] -> LISA-frame physical parameters."""
    th = np.asarray(th, dtype=np.float64)
    out = th.copy()
    tL, lamL, betaL, psiL = ssb_to_lisa(t0 + th[..., 10], th[..., 7], th[..., 8], th[..., 9])
    out[..., 7], out[..., 8], out[..., 9], out[..., 10] = lamL, betaL, psiL, tL - t0
    return out


def lisa_to_physical(thL, t0):
    """LISA-frame physical parameters [..., 11] -> SSB physical parameters."""
    thL = np.asarray(thL, dtype=np.float64)
    out = thL.copy()
    t, lam, beta, psi = lisa_to_ssb(t0 + thL[..., 10], thL[..., 7], thL[..., 8], thL[..., 9])
    out[..., 7], out[..., 8], out[..., 9], out[..., 10] = lam, beta, psi, t - t0
    return out


def to_sampling_lisa(thL):
    thL = np.asarray(thL, dtype=np.float64)
    x = np.empty_like(thL)
    x[..., 0] = np.log(thL[..., 0])
    x[..., 1:4] = thL[..., 1:4]
    x[..., 4] = np.log(thL[..., 4])
    x[..., 5] = thL[..., 5]
    x[..., 6] = np.cos(thL[..., 6])
    x[..., 7] = thL[..., 7]
    x[..., 8] = np.sin(thL[..., 8])
    x[..., 9] = thL[..., 9]
    x[..., 10] = thL[..., 10]
    return x


def from_sampling_lisa(x):
    x = np.asarray(x, dtype=np.float64)
    th = np.empty_like(x)
    th[..., 0] = np.exp(x[..., 0])
    th[..., 1:4] = x[..., 1:4]
    th[..., 4] = np.exp(x[..., 4])
    th[..., 5] = x[..., 5]
    th[..., 6] = np.arccos(np.clip(x[..., 6], -1.0, 1.0))
    th[..., 7] = x[..., 7]
    th[..., 8] = np.arcsin(np.clip(x[..., 8], -1.0, 1.0))
    th[..., 9] = x[..., 9]
    th[..., 10] = x[..., 10]
    return th


def sampling_lisa_to_ssb(x, t0):
    """LISA-frame sampling coordinates -> SSB physical parameters."""
    return lisa_to_physical(from_sampling_lisa(x), t0)


def _ssb_sampling_of_lisa(x, t0):
    th = sampling_lisa_to_ssb(x, t0)
    with np.errstate(invalid="ignore", divide="ignore"):
        return inputs.to_sampling(th)


def log_jacobian(x, t0, h=(1e-7, 1e-7, 1e-7, 1e-3)):
    """ln |d(lambda, sin beta, psi, ln t_ref) / d(lambda_L, sin beta_L, psi_L,
    tau_L)| at LISA-frame sampling coordinates x[..., 11], by central
    differences (the map is smooth; steps well inside its scales)."""
    x = np.asarray(x, dtype=np.float64)
    cols = (7, 8, 9, 10)
    J = np.empty(x.shape[:-1] + (4, 4))
    for j, (c, hj) in enumerate(zip(cols, h)):
        xp, xm = x.copy(), x.copy()
        xp[..., c] += hj
        xm[..., c] -= hj
        yp, ym = _ssb_sampling_of_lisa(xp, t0), _ssb_sampling_of_lisa(xm, t0)
        d = (yp - ym)[..., cols]
        # longitudes and polarisation angles are periodic
        d[..., 0] = np.mod(d[..., 0] + math.pi, 2.0 * math.pi) - math.pi
        d[..., 2] = np.mod(d[..., 2] + 0.5 * math.pi, math.pi) - 0.5 * math.pi
        J[..., :, j] = d / (2.0 * hj)
    with np.errstate(divide="ignore"):
        return np.log(np.abs(np.linalg.det(J)))


def lisa_logprior(t0, lo=inputs.PRIOR_LO, hi=inputs.PRIOR_HI):
    """The Table I prior (uniform in the SSB sampling coordinates) carried to
    the LISA-frame sampling coordinates: ln pi_SSB(x_SSB(x)) + ln |J|.
    Outside the LISA-frame angle ranges (lambda_L in [0, 2 pi), sin beta_L
    in [-1, 1], psi_L in [0, pi)) it is -inf, so each point is counted once."""
    lo = np.asarray(lo)
    hi = np.asarray(hi)

    def lp(x):
        x = np.atleast_2d(np.asarray(x, dtype=np.float64))
        ok = ((x[:, 7] >= 0.0) & (x[:, 7] < 2.0 * math.pi) & (np.abs(x[:, 8]) <= 1.0) &
              (x[:, 9] >= 0.0) & (x[:, 9] < math.pi))
        out = np.full(len(x), -np.inf)
        if ok.any():
            xs = _ssb_sampling_of_lisa(x[ok], t0)
            inside = np.all((xs >= lo) & (xs <= hi), axis=-1)
            val = np.where(inside, log_jacobian(x[ok], t0), -np.inf)
            out[ok] = val
        return out
    return lp


def sky_modes(thL):
    """The eight LISA-frame sky modes of LISA-frame physical parameters
    thL[11] (Sec. III.B): longitudes lambda_L + k pi/2 (k = 0..3), each
    above and below the constellation plane.  Returns [8][11], mode 0 the
    input.  With the rotation, psi_L moves by k pi/2; with the reflection,
    beta_L -> -beta_L, psi_L -> pi - psi_L and iota -> pi - iota (the maps
    under which the response is unchanged, see the module notes)."""
    thL = np.asarray(thL, dtype=np.float64)
    out = []
    for refl in (False, True):
        for k in range(4):
            m = thL.copy()
            m[7] = np.mod(thL[7] + k * 0.5 * math.pi, 2.0 * math.pi)
            m[9] = np.mod(thL[9] + k * 0.5 * math.pi, math.pi)
            if refl:
                m[8] = -thL[8]
                m[9] = np.mod(math.pi - m[9], math.pi)
                m[6] = math.pi - thL[6]
            out.append(m)
    return np.stack(out)


def sky_mode_walkers(thL, n_temps: int, per_mode: int, rel: float, seed: int):
    """Initial LISA-frame sampling coordinates [n_temps][8 * per_mode][11]:
    per temperature, per_mode walkers in a small Gaussian ball (relative
    width rel, as inputs.ball) about each of the eight sky modes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    modes = to_sampling_lisa(sky_modes(thL))               # [8][11]
    x = np.repeat(modes[None, :, None, :], n_temps, axis=0)
    x = np.repeat(x, per_mode, axis=2)                      # [T][8][per_mode][11]
    scale = rel * np.maximum(np.abs(modes), 1e-3)
    x = x + scale[None, :, None, :] * rng.standard_normal(x.shape)
    x[..., 7] = np.mod(x[..., 7], 2.0 * math.pi)
    x[..., 8] = np.clip(x[..., 8], -1.0, 1.0)
    x[..., 9] = np.mod(x[..., 9], math.pi)
    return x.reshape(n_temps, 8 * per_mode, 11)
