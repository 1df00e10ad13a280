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
