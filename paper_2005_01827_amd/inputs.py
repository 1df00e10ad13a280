"""Seeded synthetic inputs shaped like the workloads of arXiv:2005.01827.

This module holds no step of the likelihood itself.  It provides what both the
HIP path and the CPU oracle consume as *inputs*: the frequency grid, an
analytic LISA-like noise PSD, Gaussian frequency-domain noise, luminosity
distance from redshift, the Table I prior box and its sampling coordinates,
and seeded walker batches.  Every random draw uses numpy's PCG64 with an
explicit seed.

Readings of the paper used here (each is listed in the design notes):
  * grid: f_k = k df with df = 1/T_obs, bins k0..k0+n-1 (Sec. II, Eq. innerprod
    discretised as a rectangle rule);
  * noise (Sec. II, Eq. noise_gen): real and imaginary parts iid normal with
    standard deviation sqrt(S_n / (4 df)), so that E|n|^2 = S_n / (2 df), the
    one-sided convention that makes E<n|n>_c = 2 per bin;
  * PSD (Sec. II names SciRDv1 + a Galactic foreground through the LDC ``tdi``
    package, which is not available): an analytic acceleration + optical-path
    noise model propagated through first-generation TDI A, E, T;
  * D_L(z): flat LambdaCDM, H0 = 67.74 km/s/Mpc, Omega_m = 0.3075; it matches
    the distances quoted in Sec. II (Table I bounds) and Sec. IV (Table II)
    to about 0.5 %.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

C_SI = 299792458.0
LARM_M = 2.5e9
YEAR_S = 3.15576e7

MODES_ALL = ((2, 2), (3, 3), (4, 4), (2, 1), (3, 2), (4, 3))

# Table I: lower and upper bounds in sampling coordinates
# (ln M_T, q, a1, a2, ln D_L, phi_ref, cos iota, lambda, sin beta, psi, ln t_ref).
PRIOR_LO = np.array([math.log(1e3), 0.05, -0.99, -0.99, math.log(0.044), 0.0, -1.0, 0.0, -1.0, 0.0, 0.0])
PRIOR_HI = np.array([math.log(1e9), 1.0, 0.99, 0.99, math.log(1298.0), 2 * math.pi, 1.0, 2 * math.pi, 1.0,
                     math.pi, math.log(3.15576e8)])


@dataclasses.dataclass(frozen=True)
class Grid:
    """Dense frequency grid f_k = k df, k = k0 .. k0+n-1."""
    df: float
    k0: int
    n: int

    @staticmethod
    def from_band(T_obs: float, fmin: float, fmax: float) -> "Grid":
        df = 1.0 / T_obs
        k0 = int(math.ceil(fmin * T_obs))
        k1 = int(math.floor(fmax * T_obs))
        return Grid(df, k0, k1 - k0 + 1)

    @property
    def freqs(self) -> np.ndarray:
        return (self.k0 + np.arange(self.n, dtype=np.float64)) * self.df


def psd_aet(f: np.ndarray) -> np.ndarray:
    """Analytic one-sided PSD of the A, E, T channels (fractional frequency).

    Acceleration noise (3e-15 m s^-2 Hz^-1/2 with a 0.4 mHz reddening and an
    8 mHz roll-up) and optical-path noise (15 pm Hz^-1/2 with a 2 mHz
    reddening), propagated through first-generation TDI of an equal-arm
    triangle of arm L = 2.5e9 m.  Returns S[3][n] with S_A = S_E.
    """
    f = np.asarray(f, dtype=np.float64)
    x = 2.0 * math.pi * f * LARM_M / C_SI
    s_acc = (3e-15) ** 2 * (1.0 + (4e-4 / f) ** 2) * (1.0 + (f / 8e-3) ** 4)
    s_oms = (15e-12) ** 2 * (1.0 + (2e-3 / f) ** 4)
    s_pm = s_acc / (2.0 * math.pi * f * C_SI) ** 2
    s_op = s_oms * (2.0 * math.pi * f / C_SI) ** 2
    sx2 = np.sin(x) ** 2
    s_ae = 8.0 * sx2 * (2.0 * s_pm * (3.0 + 2.0 * np.cos(x) + np.cos(2.0 * x)) + s_op * (2.0 + np.cos(x)))
    sh2 = np.sin(0.5 * x) ** 2
    s_t = 32.0 * sx2 * sh2 * (4.0 * s_pm * sh2 + s_op)
    return np.stack([s_ae, s_ae, s_t])


def noise(grid: Grid, psd: np.ndarray, seed: int) -> np.ndarray:
    """Gaussian frequency-domain noise n[3][n] (complex128)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sig = np.sqrt(psd / (4.0 * grid.df))
    return sig * rng.standard_normal(psd.shape) + 1j * (sig * rng.standard_normal(psd.shape))


def luminosity_distance_gpc(z: float, H0: float = 67.74, Om: float = 0.3075) -> float:
    """Flat LambdaCDM luminosity distance in Gpc (composite Simpson rule)."""
    nint = 4096
    zz = np.linspace(0.0, z, nint + 1)
    inv_e = 1.0 / np.sqrt(Om * (1.0 + zz) ** 3 + (1.0 - Om))
    h = z / nint
    integral = h / 3.0 * (inv_e[0] + inv_e[-1] + 4.0 * inv_e[1:-1:2].sum() + 2.0 * inv_e[2:-1:2].sum())
    dh_gpc = C_SI / 1e3 / H0 / 1e3
    return (1.0 + z) * dh_gpc * integral


def to_physical(x: np.ndarray) -> np.ndarray:
    """Sampling coordinates -> physical parameters (M_T, q, a1, a2, D_L[Gpc],
    phi_ref, iota, lambda, beta, psi, t_ref[s]), last axis of length 11."""
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
    th[..., 10] = np.exp(x[..., 10])
    return th


def to_sampling(th: np.ndarray) -> np.ndarray:
    th = np.asarray(th, dtype=np.float64)
    x = np.empty_like(th)
    x[..., 0] = np.log(th[..., 0])
    x[..., 1:4] = th[..., 1:4]
    x[..., 4] = np.log(th[..., 4])
    x[..., 5] = th[..., 5]
    x[..., 6] = np.cos(th[..., 6])
    x[..., 7] = th[..., 7]
    x[..., 8] = np.sin(th[..., 8])
    x[..., 9] = th[..., 9]
    x[..., 10] = np.log(th[..., 10])
    return x


def in_prior(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x)
    return np.all((x >= PRIOR_LO) & (x <= PRIOR_HI), axis=-1)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    grid: Grid
    t0: float
    injection: np.ndarray          # physical parameters [11]
    walkers: np.ndarray            # physical parameters [B][11]
    modes: tuple = MODES_ALL
    ns: int = 256
    noise_seed: int | None = None


def _uniform_extrinsics(rng) -> np.ndarray:
    """phi_ref, iota, lambda, beta, psi drawn uniform in their Table I coordinates."""
    lo, hi = PRIOR_LO[5:10], PRIOR_HI[5:10]
    x = lo + (hi - lo) * rng.random(5)
    return np.array([x[0], math.acos(x[1]), x[2], math.asin(x[3]), x[4]])


def ball(center: np.ndarray, n: int, rel: float, seed: int) -> np.ndarray:
    """n walkers from a Gaussian ball in sampling coordinates, sigma_i = rel*|x_i|,
    returned as physical parameters, clipped into the prior box."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xc = to_sampling(center)
    x = xc + rel * np.abs(xc) * rng.standard_normal((n, 11))
    x = np.clip(x, PRIOR_LO, PRIOR_HI)
    return to_physical(x)


def short_grid(n_walkers: int = 1) -> Workload:
    """Batch-1 latency case: T_obs = 2^22 s, f in [1e-4, 3e-2] Hz."""
    T = 2.0 ** 22
    grid = Grid.from_band(T, 1e-4, 3e-2)
    rng = np.random.Generator(np.random.PCG64(1))
    ext = _uniform_extrinsics(rng)
    inj = np.array([1e6, 0.2, 0.3, -0.2, luminosity_distance_gpc(2.0), *ext, 50.25])
    walkers = inj[None, :].copy() if n_walkers == 1 else ball(inj, n_walkers, 1e-3, 11)
    return Workload(f"{n_walkers}walkers-Tobs2^22", grid, 0.9 * T, inj, walkers, noise_seed=101)


def year_grid(n_walkers: int = 1024) -> Workload:
    """Throughput case: 1024 walkers, T_obs = 2^25 s, f in [1e-5, 0.1] Hz."""
    T = 2.0 ** 25
    grid = Grid.from_band(T, 1e-5, 0.1)
    inj = np.array([3e6, 0.3, 0.3, -0.2, luminosity_distance_gpc(3.0), 2.14, 1.05, 2 * math.pi - 0.024,
                    0.62, 2.03, 50.25])
    walkers = ball(inj, n_walkers, 1e-3, 202)
    return Workload(f"{n_walkers}walkers-Tobs2^25", grid, YEAR_S, inj, walkers, noise_seed=2002)


def uneven_batch(n_walkers: int = 2048) -> Workload:
    """Uneven batch: log-uniform M_T in [1e5, 1e8], q ~ U[0.1,1], spins ~ U[-0.99,0.99],
    z ~ U[1,10], other parameters uniform over Table I; config-2 grid and data."""
    base = year_grid(1)
    rng = np.random.Generator(np.random.PCG64(3))
    w = np.empty((n_walkers, 11))
    w[:, 0] = np.exp(rng.uniform(math.log(1e5), math.log(1e8), n_walkers))
    w[:, 1] = rng.uniform(0.1, 1.0, n_walkers)
    w[:, 2] = rng.uniform(-0.99, 0.99, n_walkers)
    w[:, 3] = rng.uniform(-0.99, 0.99, n_walkers)
    zs = rng.uniform(1.0, 10.0, n_walkers)
    w[:, 4] = [luminosity_distance_gpc(z) for z in zs]
    for i in range(n_walkers):
        w[i, 5:10] = _uniform_extrinsics(rng)
    w[:, 10] = np.exp(rng.uniform(PRIOR_LO[10], PRIOR_HI[10], n_walkers))
    return Workload(f"uneven-{n_walkers}walkers-Tobs2^25", base.grid, base.t0, base.injection, w,
                    noise_seed=base.noise_seed)


def table2_binaries() -> dict:
    """Injection parameters of the seven test binaries of Sec. IV (Table II),
    as physical parameters [11] keyed by binary number.

    The table prints rounded values, used as printed; q is taken as the
    fraction it names (1/3, 1/5, 7/10).  A negative ecliptic longitude is
    mapped into the prior range [0, 2 pi).  t_ref is relative to t0 = 1 yr,
    as for the other workloads on the 2^25-s grid.  Binaries 2 and 3 repeat
    Binary 1 (2 has no noise; 3 keeps the spins fixed while sampling).
    """
    b13 = [2e6, 1.0 / 3.0, 0.0, 0.0, 36.59, 2.14, 1.05, -0.024, 0.62, 2.03, 50.25]
    rows = {
        1: b13, 2: b13, 3: b13,
        4: [2e6, 1.0 / 3.0, 0.85, 0.88, 36.59, 2.14, 1.05, -0.024, 0.62, 2.03, 50.25],
        5: [2e6, 1.0 / 3.0, -0.83, -0.89, 36.59, 2.14, 1.05, -0.024, 0.62, 2.03, 50.25],
        6: [4e7, 1.0 / 5.0, 0.0, 0.0, 15.93, 3.10, 1.34, 4.21, -0.73, 0.14, 23.93],
        7: [3e5, 7.0 / 10.0, 0.0, 0.0, 70.58, 1.22, 1.32, 2.24, -0.22, 2.73, 94.33],
    }
    out = {}
    for b, r in rows.items():
        th = np.array(r, dtype=np.float64)
        th[7] = th[7] % (2.0 * math.pi)
        out[b] = th
    return out


def table2_workload(binary: int) -> Workload:
    """One Table II binary on the 2^25-s grid (f in [1e-5, 0.1] Hz, t0 = 1 yr);
    the single walker sits on the injection.  Binaries 2 and 7 were injected
    without noise in Sec. IV; the others carry a noise seed."""
    base = year_grid(1)
    inj = table2_binaries()[binary]
    seed = None if binary in (2, 7) else 7000 + binary
    return Workload(f"binary{binary}-Tobs2^25", base.grid, base.t0, inj, inj[None, :].copy(), noise_seed=seed)


def small_config(n_walkers: int = 8, seed: int = 7) -> Workload:
    """A small grid the oracle finishes in well under a second per walker:
    T_obs = 2^20 s, f in [2e-4, 2e-2] Hz, M_T = 2e6, q = 1/3."""
    T = 2.0 ** 20
    grid = Grid.from_band(T, 2e-4, 2e-2)
    inj = np.array([2e6, 1.0 / 3.0, 0.2, -0.1, luminosity_distance_gpc(3.0), 2.14, 1.05, 2 * math.pi - 0.024,
                    0.62, 2.03, 50.25])
    walkers = ball(inj, n_walkers, 1e-3, seed)
    return Workload(f"small-{n_walkers}walkers-Tobs2^20", grid, 0.9 * T, inj, walkers, noise_seed=seed + 1000)


# ---------------------------------------------------------------------------
# Learned-proposal inputs: coupling-layer permutations, flat parameter arrays
# and training samples.  Sizes (parameter counts) are passed in; nothing here
# evaluates the flow.
# ---------------------------------------------------------------------------
def flow_perms(dim: int, n_layers: int, seed: int) -> np.ndarray:
    """[n_layers][dim] int32: one seeded random permutation per layer."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.permutation(dim) for _ in range(n_layers)]).astype(np.int32)


def flow_params(n_params: int, scale: float, seed: int) -> np.ndarray:
    """A flat float32 parameter array, iid uniform in [-scale, scale]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, n_params).astype(np.float32)


def banana(n: int, dim: int, seed: int, b: float = 0.6, sx: float = 2.0) -> np.ndarray:
    """n draws of a curved ('banana') density in dim >= 2 dimensions:
    x0 ~ N(0, sx^2), x1 = b (x0^2 - sx^2) + N(0, 1), others N(0, 1)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, dim))
    x[:, 0] *= sx
    x[:, 1] += b * (x[:, 0] ** 2 - sx * sx)
    return x
