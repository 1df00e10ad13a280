"""Sampler and ESS (Sec. III) on analytic targets, CPU only."""
import math
import os

import numpy as np
import pytest
from scipy import stats

from paper_2005_01827_amd import sampler as S


def test_stretch_factor_distribution():
    """Y ~ g(y) ~ y^{-1/2} on [1/a, a]: CDF F(y) = (sqrt y - a^{-1/2}) / (a^{1/2} - a^{-1/2})."""
    rng = np.random.default_rng(1)
    for a in (1.15, 2.0):
        y = S.stretch_factor(rng, a, 200000)
        assert y.min() >= 1 / a and y.max() <= a
        cdf = lambda v: (np.sqrt(v) - a ** -0.5) / (a ** 0.5 - a ** -0.5)
        assert stats.kstest(y, cdf).pvalue > 1e-3


def test_ladder():
    b = S.ladder(8)
    assert b[0] == 1.0 and b[-1] == 0.0
    assert np.allclose(1 / b[:-1], 2.04807 ** np.arange(7))


def test_ar1_integrated_time():
    """AR(1) with coefficient r: tau = (1 + r) / (1 - r)."""
    rng = np.random.default_rng(2)
    for r in (0.5, 0.9):
        n, w = 20000, 32
        x = np.zeros((n, w))
        e = rng.standard_normal((n, w)) * math.sqrt(1 - r * r)
        for i in range(1, n):
            x[i] = r * x[i - 1] + e[i]
        tau = S.integrated_time(x)
        assert abs(tau / ((1 + r) / (1 - r)) - 1) < 0.08


def _gauss_target(dim, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((dim, dim))
    cov = A @ A.T / dim + np.eye(dim) * 0.2
    mu = rng.standard_normal(dim)
    icov = np.linalg.inv(cov)

    def ll(x):
        d = np.atleast_2d(x) - mu
        return -0.5 * np.einsum("ni,ij,nj->n", d, icov, d)
    return mu, cov, ll


def test_batch_means_standard_error():
    """AR(1) walkers: the standard error of the ensemble mean is
    sqrt(tau / (N W)) per unit variance; walkers that share a common slow
    component (here one AR(1) path added to every walker) are correlated with
    each other, which the batch means see and the walker-averaged
    autocorrelation (own-mean per walker) does not."""
    rng = np.random.default_rng(7)
    r, n, w = 0.8, 20000, 32
    e = rng.standard_normal((n, w, 3))
    x = np.empty_like(e)
    x[0] = e[0]
    for t in range(1, n):
        x[t] = r * x[t - 1] + math.sqrt(1 - r * r) * e[t]
    se = S.batch_means_se(x, 40)
    want = math.sqrt((1 + r) / (1 - r) / (n * w))
    assert np.all(np.abs(se / want - 1) < 0.35), se / want
    # a shared slow drift: same AR(1) path (r = 0.999) in every walker
    c = np.empty(n)
    c[0] = 0.0
    g = rng.standard_normal(n)
    for t in range(1, n):
        c[t] = 0.999 * c[t - 1] + math.sqrt(1 - 0.999 ** 2) * g[t]
    y = x + 0.3 * c[:, None, None]
    se_y = S.batch_means_se(y, 40)
    _, tau_y, _ = S.ess(y)
    naive = np.sqrt(y.reshape(-1, 3).var(0) * tau_y / (n * w))
    assert np.all(se_y > 3 * naive)


def test_ensemble_mean_standard_error():
    """The autocorrelation estimate of the ensemble mean's standard error on
    independent AR(1) walkers, whose ensemble mean is AR(1) with the same
    coefficient: sqrt(tau / (N W)) per unit variance, tau = (1 + r) / (1 - r);
    and on walkers that share one slow AR(1) component, where it exceeds the
    walker-averaged figure as the batch means do."""
    rng = np.random.default_rng(9)
    r, n, w = 0.8, 20000, 32
    e = rng.standard_normal((n, w, 3))
    x = np.empty_like(e)
    x[0] = e[0]
    for t in range(1, n):
        x[t] = r * x[t - 1] + math.sqrt(1 - r * r) * e[t]
    se = S.ensemble_mean_se(x)
    want = math.sqrt((1 + r) / (1 - r) / (n * w))
    assert np.all(np.abs(se / want - 1) < 0.15), se / want
    c = np.empty(n)
    c[0] = 0.0
    g = rng.standard_normal(n)
    for t in range(1, n):
        c[t] = 0.99 * c[t - 1] + math.sqrt(1 - 0.99 ** 2) * g[t]
    y = x + 0.3 * c[:, None, None]
    # shared part: variance 0.09, tau = 1.99 / 0.01; own part as above
    want_y = math.sqrt((0.09 * 199.0 + (1 + r) / (1 - r) / w) / n)
    se_y = S.ensemble_mean_se(y)
    assert np.all(np.abs(se_y / want_y - 1) < 0.35), se_y / want_y


def test_stretch_move_recovers_correlated_gaussian():
    dim = 11
    mu, cov, ll = _gauss_target(dim, 3)
    flat = lambda x: np.zeros(len(np.atleast_2d(x)))
    smp = S.PTSampler(ll, flat, [1.0], 64, dim, a=2.0, seed=4)
    rng = np.random.default_rng(5)
    smp.initialize((mu + 0.1 * rng.standard_normal((64, dim)))[None])
    smp.run(1500)
    chain = smp.run(6000)                        # [N][W][D]
    flat_s = chain.reshape(-1, dim)
    n_eff, tau, _ = S.ess(chain)
    se = np.sqrt(np.diag(cov) / n_eff)
    assert np.all(np.abs(flat_s.mean(0) - mu) < 5 * se)
    assert np.allclose(np.cov(flat_s.T), cov, atol=0.15 * np.abs(cov).max())
    acc = smp.state.accepted[0] / smp.state.proposed[0]
    assert 0.1 < acc < 0.9


def test_parallel_tempering_bimodal_weights():
    """Two well-separated Gaussians with weights 0.3 / 0.7: the T = 1 chain
    must find both and weight them correctly."""
    dim = 2
    c1, c2 = np.array([-5.0, 0.0]), np.array([5.0, 0.0])

    def ll(x):
        x = np.atleast_2d(x)
        l1 = np.log(0.3) - 0.5 * np.sum((x - c1) ** 2, axis=1)
        l2 = np.log(0.7) - 0.5 * np.sum((x - c2) ** 2, axis=1)
        return np.logaddexp(l1, l2)
    lp = S.box_logprior([-20, -20], [20, 20])
    betas = S.ladder(6, ratio=2.5)
    smp = S.PTSampler(ll, lp, betas, 32, dim, a=2.0, seed=6)
    rng = np.random.default_rng(7)
    x0 = np.tile(c1, (len(betas), 32, 1)) + 0.1 * rng.standard_normal((len(betas), 32, dim))
    smp.initialize(x0)                           # everything starts in the light mode
    smp.run(1000)
    chain = smp.run(6000, thin=2)
    frac = np.mean(chain[..., 0] > 0)
    assert abs(frac - 0.7) < 0.06
    assert np.all(smp.state.swaps_accepted > 0)


def test_independence_proposal_with_exact_density():
    """With q equal to the target, every independence proposal is accepted."""
    dim = 5
    mu, cov, ll = _gauss_target(dim, 8)
    chol = np.linalg.cholesky(cov)
    icov = np.linalg.inv(cov)
    lognorm = -0.5 * (dim * math.log(2 * math.pi) + np.linalg.slogdet(cov)[1])

    class Exact:
        def sample(self, n, rng):
            z = rng.standard_normal((n, dim))
            x = mu + z @ chol.T
            return x, self.logq(x)

        def logq(self, x):
            d = np.atleast_2d(x) - mu
            return lognorm - 0.5 * np.einsum("ni,ij,nj->n", d, icov, d)

    flat = lambda x: np.zeros(len(np.atleast_2d(x)))
    smp = S.PTSampler(ll, flat, [1.0], 32, dim, seed=9, proposal=Exact(), p_flow=1.0)
    smp.initialize(mu[None, None] + np.zeros((1, 32, dim)))
    chain = smp.run(800)
    assert smp.state.flow_proposed > 0 and smp.state.flow_accepted == smp.state.flow_proposed
    n_eff, tau, _ = S.ess(chain)
    assert tau < 2.0
    assert np.allclose(chain.reshape(-1, dim).mean(0), mu, atol=0.1)


def test_checkpoint_resume_is_bit_identical(tmp_path):
    dim = 4
    mu, cov, ll = _gauss_target(dim, 10)
    flat = lambda x: np.zeros(len(np.atleast_2d(x)))
    betas = S.ladder(3)

    def fresh():
        s = S.PTSampler(ll, flat, betas, 16, dim, seed=11)
        s.initialize(mu + np.random.default_rng(12).standard_normal((3, 16, dim)) * 0.1)
        return s
    a = fresh()
    a.run(50)
    path = os.path.join(tmp_path, "ckpt.npz")
    a.save(path)
    tail_a = a.run(40)
    b = S.PTSampler(ll, flat, betas, 16, dim, seed=999)
    b.load(path)
    tail_b = b.run(40)
    assert np.array_equal(tail_a, tail_b)
    assert np.array_equal(a.state.logl, b.state.logl)


# ---------------------------------------------------------------------------
# Thermodynamic-integration evidence, adaptive tempering, fixed coordinates
# ---------------------------------------------------------------------------
D_BOX, SIG_BOX, A_BOX = 2, 0.5, 5.0


def _box_gauss():
    """Isotropic Gaussian likelihood exp(-|x|^2 / (2 sig^2)) under a uniform
    prior on [-a, a]^D: Z = (sig sqrt(2 pi) erf(a / (sig sqrt 2)) / (2a))^D."""
    def ll(x):
        return -0.5 * np.sum(np.atleast_2d(x) ** 2, axis=1) / SIG_BOX ** 2

    def lp(x):
        x = np.atleast_2d(x)
        return np.where(np.all(np.abs(x) <= A_BOX, axis=1), 0.0, -np.inf)
    lnz = D_BOX * math.log(SIG_BOX * math.sqrt(2 * math.pi) * math.erf(A_BOX / (SIG_BOX * math.sqrt(2))) / (2 * A_BOX))
    return ll, lp, lnz


def _box_gauss_mean_logl(beta):
    """<ln L> under L^beta pi: each coordinate is a normal of scale sig/sqrt(beta)
    truncated to [-a, a], whose second moment is s^2 (1 - 2 c phi(c) / (2 Phi(c) - 1)),
    c = a / s; at beta = 0 the prior's a^2 / 3."""
    if beta == 0.0:
        ex2 = A_BOX ** 2 / 3
    else:
        s = SIG_BOX / math.sqrt(beta)
        c = A_BOX / s
        ex2 = s * s * (1 - 2 * c * stats.norm.pdf(c) / (2 * stats.norm.cdf(c) - 1))
    return -D_BOX * ex2 / (2 * SIG_BOX ** 2)


def test_ti_evidence_quadrature_converges_to_closed_form():
    _, _, exact = _box_gauss()
    errs = []
    for nr, ratio in ((21, 2.0), (30, 1.5), (60, 1.2)):
        b = S.ladder(nr, ratio)
        lnz, est = S.ti_evidence(b, [_box_gauss_mean_logl(x) for x in b])
        errs.append(abs(lnz - exact))
        assert errs[-1] < est, (nr, lnz, exact, est)
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.02
    # the ladder's order does not matter; it must span beta = 0 .. 1
    b = S.ladder(30, 1.5)
    m = [_box_gauss_mean_logl(x) for x in b]
    assert S.ti_evidence(b[::-1], m[::-1])[0] == S.ti_evidence(b, m)[0]
    with pytest.raises(ValueError):
        S.ti_evidence(S.ladder(5, top_infinite=False), np.zeros(5))


def test_parallel_tempering_evidence_matches_closed_form():
    ll, lp, exact = _box_gauss()
    betas = S.ladder(30, 1.5)
    smp = S.PTSampler(ll, lp, betas, 32, D_BOX, a=2.0, seed=3, record_logl=True)
    smp.initialize(np.random.default_rng(4).uniform(-A_BOX, A_BOX, (30, 32, D_BOX)))
    smp.run(300)
    smp.logl_history.clear()
    smp.run(1500)
    lnz, est = S.ti_evidence(smp.betas, np.mean(np.array(smp.logl_history), axis=(0, 2)))
    quad, _ = S.ti_evidence(betas, [_box_gauss_mean_logl(x) for x in betas])
    assert abs(lnz - quad) < 0.05           # Monte Carlo part: the chains' <ln L>_beta
    assert abs(lnz - exact) < est + 0.05    # and the whole estimate, within its quadrature error


def test_adapt_ladder_rule():
    b = S.ladder(6)
    # equal acceptances: the ladder does not move
    assert np.array_equal(S.adapt_ladder(b, np.full(5, 0.4), 0, 100.0, 10.0), b)
    A = np.array([0.9, 0.3, 0.5, 0.5, 0.2])
    nb = S.adapt_ladder(b, A, 50, 100.0, 10.0)
    kappa = 100.0 / 150.0 / 10.0
    T, nT = 1 / b[:-1], 1 / nb[:-1]
    assert nb[0] == 1.0 and nb[-1] == 0.0 and np.all(np.diff(nb) < 0)
    assert np.allclose(np.diff(nT) / np.diff(T), np.exp(kappa * (A[:-1] - A[1:])), rtol=1e-13)
    with pytest.raises(ValueError):
        S.PTSampler(lambda x: x[:, 0], lambda x: 0 * x[:, 0], S.ladder(4, top_infinite=False), 8, 2, adapt=True)


def test_adaptive_tempering_evens_swap_acceptance(tmp_path):
    ll, lp, _ = _box_gauss()
    spread = {}
    for adapt in (False, True):
        smp = S.PTSampler(ll, lp, S.ladder(10), 32, D_BOX, a=2.0, seed=5, adapt=adapt, adapt_lag=1000,
                          adapt_time=20)
        smp.initialize(np.random.default_rng(6).uniform(-A_BOX, A_BOX, (10, 32, D_BOX)))
        smp.run(2000)
        smp.adapt = False
        a0, p0 = smp.state.swaps_accepted.copy(), smp.state.swaps_proposed.copy()
        smp.run(1000)
        fr = (smp.state.swaps_accepted - a0) / (smp.state.swaps_proposed - p0)
        spread[adapt] = fr.max() - fr.min()
        assert smp.betas[0] == 1.0 and smp.betas[-1] == 0.0 and np.all(np.diff(smp.betas) < 0)
    assert spread[True] < 0.5 * spread[False], spread
    # a checkpoint keeps the adapted ladder
    path = os.path.join(tmp_path, "adapted.npz")
    smp.save(path)
    other = S.PTSampler(ll, lp, S.ladder(10), 32, D_BOX, seed=1)
    other.load(path)
    assert np.array_equal(other.betas, smp.betas)


def test_fixed_coordinates_sample_the_conditional():
    """Holding coordinate 2 of a 3-D Gaussian fixed (as Sec. IV holds the
    spins of Binary 3) samples the conditional Gaussian of the other two."""
    dim = 3
    mu, cov, ll = _gauss_target(dim, 21)
    c = mu[2] + 0.7
    flat = lambda x: np.zeros(len(np.atleast_2d(x)))
    ll2 = S.fix_coordinates(ll, dim, {2: c})
    lp2 = S.fix_coordinates(flat, dim, {2: c})
    assert list(ll2.free) == [0, 1]
    assert np.array_equal(ll2.expand(np.array([[1.0, 2.0]])), [[1.0, 2.0, c]])
    s12 = cov[:2, 2]
    mu_c = mu[:2] + s12 * (c - mu[2]) / cov[2, 2]
    cov_c = cov[:2, :2] - np.outer(s12, s12) / cov[2, 2]
    smp = S.PTSampler(ll2, lp2, [1.0], 32, 2, a=2.0, seed=22)
    smp.initialize((mu_c + 0.1 * np.random.default_rng(23).standard_normal((32, 2)))[None])
    smp.run(500)
    chain = smp.run(4000)
    n_eff, _, _ = S.ess(chain)
    flat_s = chain.reshape(-1, 2)
    assert np.all(np.abs(flat_s.mean(0) - mu_c) < 5 * np.sqrt(np.diag(cov_c) / n_eff))
    assert np.allclose(np.cov(flat_s.T), cov_c, atol=0.1 * np.abs(cov_c).max())
    with pytest.raises(ValueError):
        ll2(np.zeros((4, 3)))


def test_curvature_covariance_and_start_on_a_gaussian():
    """For ln L = -(x - mu)^T P (x - mu)/2 the central differences are exact:
    the covariance is P^{-1} (numpy's inverse) whatever the steps; the start
    draws at temperature T have covariance T P^{-1} and lie in the prior."""
    rng = np.random.default_rng(31)
    d = 11
    A = rng.normal(size=(d, d)) / math.sqrt(d)
    P = A @ A.T + 0.5 * np.eye(d)
    P *= np.outer(np.logspace(0, 3, d), np.logspace(0, 3, d))     # widths spanning 1e3
    mu = rng.normal(size=d)

    def ll(x):
        r = np.atleast_2d(x) - mu
        return -0.5 * np.einsum("ni,ij,nj->n", r, P, r)
    cov_true = np.linalg.inv(P)
    for steps in (1e-4 * np.ones(d), np.sqrt(np.diag(cov_true))):
        C = S.curvature_covariance(ll, mu, steps)
        assert np.allclose(C, cov_true, rtol=1e-6, atol=1e-9 * np.abs(cov_true).max())
    lo, hi = mu - 50 * np.sqrt(np.diag(cov_true)), mu + 50 * np.sqrt(np.diag(cov_true))
    betas = S.ladder(3)
    x0, C = S.curvature_start(ll, S.box_logprior(lo, hi), mu, betas, 6000, seed=5, lo=lo, hi=hi)
    assert np.allclose(C, cov_true, rtol=1e-6, atol=1e-9 * np.abs(cov_true).max())
    assert x0.shape == (3, 6000, d)
    assert np.all(np.isfinite(S.box_logprior(lo, hi)(x0.reshape(-1, d))))
    for r, t in ((0, 1.0), (1, 1.0 / betas[1])):
        emp = np.cov(x0[r].T)
        # sample covariance of 6000 draws: entries within a few of their
        # standard errors, measured on the standardised scale
        s = np.sqrt(np.diag(t * cov_true))
        assert np.max(np.abs(emp / np.outer(s, s) - t * cov_true / np.outer(s, s))) < 0.08
    # a concave direction is held positive: ln L = +x0^2/2 along one axis
    def ll_saddle(x):
        x = np.atleast_2d(x)
        return 0.5 * x[:, 0] ** 2 - 0.5 * np.sum(x[:, 1:] ** 2, axis=1)
    C = S.curvature_covariance(ll_saddle, np.zeros(3), np.full(3, 1e-3))
    assert np.all(np.linalg.eigvalsh(C) > 0)
    # a flat direction is capped at a twentieth of the box; steps stay inside
    def ll_flat(x):
        x = np.atleast_2d(x)
        if np.any(np.abs(x) > 1.0):
            return np.full(len(x), -np.inf)
        return -0.5 * np.sum(x[:, 1:] ** 2 / 1e-4, axis=1)
    _, C = S.curvature_start(ll_flat, S.box_logprior(-np.ones(3), np.ones(3)), np.zeros(3), [1.0], 8, seed=1,
                             lo=-np.ones(3), hi=np.ones(3))
    assert abs(math.sqrt(C[0, 0]) - 0.1) < 1e-12 and abs(C[1, 1] - 1e-4) < 1e-10
