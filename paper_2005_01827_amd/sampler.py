"""Ensemble samplers of Sec. III of arXiv:2005.01827, driving the batched
likelihood.

* Stretch move (Sec. III.A, Goodman & Weare): walker k moves to
  theta_j + Y (theta_k - theta_j) with theta_j drawn from the complementary
  half of the ensemble and Y from g(y) ~ y^{-1/2} on [1/a, a]; it is accepted
  with probability min(1, Y^{D-1} L'/L) (tempered: (L'/L)^beta, and the prior
  ratio).  Each rung updates its two halves in turn, so one half is one
  batched likelihood call over every rung.
* Parallel tempering (Sec. III.B): rungs at temperatures T_i with
  likelihood L^{1/T_i}; after every step, walkers of adjacent rungs are paired
  at random and swapped with probability min(1, (L_i/L_j)^{beta_j - beta_i}).
  The top rung may have T = infinity (beta = 0), which samples the prior.
* Independence proposal (the learned part): with probability p_flow a
  walker's proposal is a draw x' ~ q from a trained density q instead of a
  stretch move, accepted with the Metropolis-Hastings ratio of Sec. III.A,
  min(1, (L'/L)^beta pi'/pi q(x)/q(x')).
* Autocorrelation and effective sample size (Sec. III.C): the normalized
  autocorrelation rho_f(tau) = c_f(tau)/c_f(0), c_f averaged over walkers,
  the integrated time tau_f(M) = 1 + 2 sum_{t<=M} rho_f(t) with the smallest
  window M >= 5 tau_f(M), and ESS = N / tau_f (tau_f taken as the largest
  over parameters).

Everything here runs on the host in numpy; the likelihood calls go to the
GPU through ``mbh.Likelihood`` (or any callable with the same contract).
"""
from __future__ import annotations

import dataclasses
import math
import os
import tempfile
import time
from typing import Callable, Optional

import numpy as np

from . import inputs

# ---------------------------------------------------------------------------
# Stretch-move variates
# ---------------------------------------------------------------------------


def stretch_factor(rng: np.random.Generator, a: float, size) -> np.ndarray:
    """Draws of Y with density g(y) ~ y^{-1/2} on [1/a, a] (inverse CDF:
    Y = ((a - 1) u + 1)^2 / a)."""
    u = rng.random(size)
    return ((a - 1.0) * u + 1.0) ** 2 / a


def ladder(n_rungs: int, ratio: float = 2.04807, top_infinite: bool = True) -> np.ndarray:
    """Inverse temperatures: T_k = ratio^k for the finite rungs (Sec. III.B
    uses ratio 2.04807 for D = 11), optionally with T = infinity on top."""
    n_fin = n_rungs - 1 if top_infinite else n_rungs
    T = ratio ** np.arange(n_fin, dtype=np.float64)
    betas = 1.0 / T
    if top_infinite:
        betas = np.append(betas, 0.0)
    return betas


# ---------------------------------------------------------------------------
# Autocorrelation (Sec. III.C)
# ---------------------------------------------------------------------------


def autocorr_function(chain: np.ndarray) -> np.ndarray:
    """rho_f(tau) for tau = 0..N-1 of chain[N, W] (one parameter, W walkers):
    c_f(tau) = 1/(N - tau) sum_n (f_n - mu)(f_{n+tau} - mu) per walker,
    averaged over walkers, then normalised by c_f(0)."""
    x = np.asarray(chain, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    n = x.shape[0]
    x = x - x.mean(axis=0, keepdims=True)
    nfft = 1 << (2 * n - 1).bit_length()
    f = np.fft.rfft(x, n=nfft, axis=0)
    acov = np.fft.irfft(f * np.conj(f), n=nfft, axis=0)[:n]      # sum_n x_n x_{n+tau}
    acov /= (n - np.arange(n))[:, None]
    c = acov.mean(axis=1)
    return c / c[0]


def integrated_time(chain: np.ndarray, c_window: float = 5.0) -> float:
    """tau_f with the smallest window M such that M >= c tau_f(M)."""
    rho = autocorr_function(chain)
    taus = 2.0 * np.cumsum(rho) - 1.0          # tau(M) = 1 + 2 sum_{t=1}^{M} rho(t)
    m = np.arange(len(taus))
    ok = m >= c_window * taus
    M = int(np.argmax(ok)) if ok.any() else len(taus) - 1
    return float(taus[M])


def ess(chain: np.ndarray, c_window: float = 5.0):
    """Effective sample size of chain[N, W, D]: N W / max_d tau_d.
    Returns (ess, tau_max, taus)."""
    chain = np.asarray(chain)
    n, w, d = chain.shape
    taus = np.array([integrated_time(chain[:, :, i], c_window) for i in range(d)])
    tau = float(taus.max())
    return n * w / tau, tau, taus


# ---------------------------------------------------------------------------
# Parallel-tempered ensemble sampler
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class PTState:
    x: np.ndarray            # [T][W][D] sampling coordinates
    logl: np.ndarray         # [T][W]
    logp: np.ndarray         # [T][W]
    step: int
    rng_state: dict
    accepted: np.ndarray     # [T] stretch/flow acceptances
    proposed: np.ndarray     # [T]
    swaps_accepted: np.ndarray   # [T-1]
    swaps_proposed: np.ndarray   # [T-1]
    flow_accepted: int = 0
    flow_proposed: int = 0


class PTSampler:
    """Parallel-tempered affine-invariant ensemble sampler.

    loglike: callable mapping sampling coordinates x[N][D] to ln L[N]
      (the GPU likelihood composed with inputs.to_physical, or any test
      density); called once per half-step with all rungs batched.
    logprior: callable x[N][D] -> ln prior (-inf outside the support).
    proposal: optional independence proposal with .sample(n, rng) -> (x, logq)
      and .logq(x) -> logq; used with probability p_flow at beta > 0 rungs.
    """

    def __init__(self, loglike: Callable, logprior: Callable, betas, n_walkers: int, dim: int,
                 a: float = 1.15, seed: int = 0, proposal=None, p_flow: float = 0.0):
        if n_walkers % 2 or n_walkers < 4:
            raise ValueError("n_walkers must be even and >= 4")
        self.loglike = loglike
        self.logprior = logprior
        self.betas = np.asarray(betas, dtype=np.float64)
        self.nt = len(self.betas)
        self.nw = n_walkers
        self.dim = dim
        self.a = a
        self.rng = np.random.Generator(np.random.PCG64(seed))
        self.proposal = proposal
        self.p_flow = p_flow
        self.state: Optional[PTState] = None
        self.n_like_calls = 0
        self.like_seconds = 0.0

    # -- likelihood in batches ------------------------------------------
    def _eval(self, x):
        """ln prior and ln L for x[N][D]; ln L only where the prior is finite."""
        lp = np.asarray(self.logprior(x), dtype=np.float64)
        ll = np.full(len(x), -np.inf)
        ok = np.isfinite(lp)
        if ok.any():
            t0 = time.perf_counter()
            ll[ok] = np.asarray(self.loglike(x[ok]), dtype=np.float64)
            self.like_seconds += time.perf_counter() - t0
            self.n_like_calls += 1
        return lp, ll

    def initialize(self, x0: np.ndarray):
        """x0[T][W][D] initial positions."""
        x0 = np.array(x0, dtype=np.float64)
        assert x0.shape == (self.nt, self.nw, self.dim)
        lp, ll = self._eval(x0.reshape(-1, self.dim))
        self.state = PTState(x=x0, logl=ll.reshape(self.nt, self.nw), logp=lp.reshape(self.nt, self.nw), step=0,
                             rng_state=self.rng.bit_generator.state, accepted=np.zeros(self.nt, np.int64),
                             proposed=np.zeros(self.nt, np.int64), swaps_accepted=np.zeros(max(self.nt - 1, 0), np.int64),
                             swaps_proposed=np.zeros(max(self.nt - 1, 0), np.int64))
        return self.state

    # -- one step: two half-updates and the swaps -------------------------
    def step(self):
        st = self.state
        half = self.nw // 2
        for h in (0, 1):
            act = np.arange(h * half, (h + 1) * half)
            oth = np.arange((1 - h) * half, (2 - h) * half)
            xa = st.x[:, act]                                    # [T][half][D]
            partners = self.rng.integers(0, half, size=(self.nt, half))
            xj = np.take_along_axis(st.x[:, oth], partners[..., None], axis=1)
            Y = stretch_factor(self.rng, self.a, (self.nt, half))
            prop = xj + Y[..., None] * (xa - xj)
            log_corr = (self.dim - 1) * np.log(Y)                # stretch-move Jacobian term
            use_flow = np.zeros((self.nt, half), bool)
            if self.proposal is not None and self.p_flow > 0.0:
                use_flow = (self.rng.random((self.nt, half)) < self.p_flow) & (self.betas[:, None] > 0.0)
                nf = int(use_flow.sum())
                if nf:
                    xf, lq_new = self.proposal.sample(nf, self.rng)
                    lq_old = self.proposal.logq(xa[use_flow])
                    prop[use_flow] = xf
                    log_corr[use_flow] = lq_old - lq_new      # q(x)/q(x') for an independence proposal
            lp, ll = self._eval(prop.reshape(-1, self.dim))
            lp = lp.reshape(self.nt, half)
            ll = ll.reshape(self.nt, half)
            cur_ll, cur_lp = st.logl[:, act], st.logp[:, act]
            with np.errstate(invalid="ignore"):
                dl = np.where(self.betas[:, None] > 0.0, self.betas[:, None] * (ll - cur_ll), 0.0)
                log_acc = log_corr + dl + (lp - cur_lp)
            log_acc = np.where(np.isfinite(lp) & np.isfinite(ll), log_acc, -np.inf)
            accept = np.log(self.rng.random((self.nt, half))) < log_acc
            idx = np.nonzero(accept)
            st.x[idx[0], act[idx[1]]] = prop[idx]
            st.logl[idx[0], act[idx[1]]] = ll[idx]
            st.logp[idx[0], act[idx[1]]] = lp[idx]
            st.accepted += accept.sum(axis=1)
            st.proposed += half
            st.flow_accepted += int((accept & use_flow).sum())
            st.flow_proposed += int(use_flow.sum())
        self._swap()
        st.step += 1
        st.rng_state = self.rng.bit_generator.state
        return st

    def _swap(self):
        """Swap adjacent rungs, hottest pair first, each walker paired with a
        random walker of the neighbouring rung."""
        st = self.state
        for i in range(self.nt - 1, 0, -1):
            bi, bj = self.betas[i], self.betas[i - 1]
            perm_i = self.rng.permutation(self.nw)
            perm_j = self.rng.permutation(self.nw)
            li, lj = st.logl[i, perm_i], st.logl[i - 1, perm_j]
            with np.errstate(invalid="ignore"):
                log_a = (bj - bi) * (li - lj)
            log_a = np.where(np.isfinite(log_a), log_a, -np.inf)
            acc = np.log(self.rng.random(self.nw)) < log_a
            a_i, a_j = perm_i[acc], perm_j[acc]
            for arr in (st.x, st.logl, st.logp):
                tmp = arr[i, a_i].copy()
                arr[i, a_i] = arr[i - 1, a_j]
                arr[i - 1, a_j] = tmp
            st.swaps_accepted[i - 1] += int(acc.sum())
            st.swaps_proposed[i - 1] += self.nw

    def run(self, n_steps: int, thin: int = 1, callback=None):
        """Run n_steps; return the T = 1 chain [n_steps/thin][W][D]."""
        out = []
        for s in range(n_steps):
            self.step()
            if s % thin == 0:
                out.append(self.state.x[0].copy())
            if callback is not None:
                callback(self)
        return np.array(out)

    # -- checkpoint / resume ---------------------------------------------
    def save(self, path: str):
        """Atomic checkpoint: write a temporary file, then rename it."""
        st = self.state
        d = os.path.dirname(os.path.abspath(path))
        fd, tmp = tempfile.mkstemp(dir=d, suffix=".npz")
        os.close(fd)
        import json
        np.savez(tmp, x=st.x, logl=st.logl, logp=st.logp, step=st.step, betas=self.betas,
                 accepted=st.accepted, proposed=st.proposed, swaps_accepted=st.swaps_accepted,
                 swaps_proposed=st.swaps_proposed, flow=np.array([st.flow_accepted, st.flow_proposed]),
                 rng=np.frombuffer(json.dumps(self.rng.bit_generator.state).encode(), dtype=np.uint8))
        os.replace(tmp, path)

    def load(self, path: str):
        import json
        z = np.load(path, allow_pickle=False)
        rng_state = json.loads(bytes(z["rng"]).decode())
        self.rng.bit_generator.state = rng_state
        fl = z["flow"]
        self.state = PTState(x=z["x"].copy(), logl=z["logl"].copy(), logp=z["logp"].copy(), step=int(z["step"]),
                             rng_state=rng_state, accepted=z["accepted"].copy(), proposed=z["proposed"].copy(),
                             swaps_accepted=z["swaps_accepted"].copy(), swaps_proposed=z["swaps_proposed"].copy(),
                             flow_accepted=int(fl[0]), flow_proposed=int(fl[1]))
        return self.state


def box_logprior(lo=inputs.PRIOR_LO, hi=inputs.PRIOR_HI):
    """Uniform prior over a box (Table I): 0 inside, -inf outside."""
    lo = np.asarray(lo)
    hi = np.asarray(hi)

    def lp(x):
        x = np.atleast_2d(x)
        inside = np.all((x >= lo) & (x <= hi), axis=-1)
        return np.where(inside, 0.0, -np.inf)
    return lp


def gpu_loglike(L):
    """ln L of sampling coordinates through an mbh.Likelihood (synchronous)."""
    import torch

    def f(x):
        th = inputs.to_physical(np.asarray(x))
        out = L.loglike(th)
        return out.cpu().numpy()
    return f
