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
                    if hasattr(self.proposal, "propose"):
                        xf, lq_new, lq_old = self.proposal.propose(xa[use_flow], self.rng)
                    else:
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
        extra = {}
        if isinstance(self.proposal, FlowProposal):
            extra = dict(flow_params=self.proposal.flow.get_params(), flow_mu=self.proposal.mu,
                         flow_sd=self.proposal.sd, p_flow=np.array(self.p_flow))
        np.savez(tmp, x=st.x, logl=st.logl, logp=st.logp, step=st.step, betas=self.betas,
                 accepted=st.accepted, proposed=st.proposed, swaps_accepted=st.swaps_accepted,
                 swaps_proposed=st.swaps_proposed, flow=np.array([st.flow_accepted, st.flow_proposed]),
                 rng=np.frombuffer(json.dumps(self.rng.bit_generator.state).encode(), dtype=np.uint8), **extra)
        os.replace(tmp, path)

    def load(self, path: str):
        import json
        z = np.load(path, allow_pickle=False)
        rng_state = json.loads(bytes(z["rng"]).decode())
        self.rng.bit_generator.state = rng_state
        fl = z["flow"]
        if "flow_params" in z.files and isinstance(self.proposal, FlowProposal):
            self.proposal.flow.set_params(z["flow_params"])
            self.proposal.mu = z["flow_mu"].copy()
            self.proposal.sd = z["flow_sd"].copy()
            self.p_flow = float(z["p_flow"])
        self.state = PTState(x=z["x"].copy(), logl=z["logl"].copy(), logp=z["logp"].copy(), step=int(z["step"]),
                             rng_state=rng_state, accepted=z["accepted"].copy(), proposed=z["proposed"].copy(),
                             swaps_accepted=z["swaps_accepted"].copy(), swaps_proposed=z["swaps_proposed"].copy(),
                             flow_accepted=int(fl[0]), flow_proposed=int(fl[1]))
        return self.state


class FlowProposal:
    """Independence proposal from the learned affine-coupling flow (mbh.Flow).

    The flow models standardized coordinates u = (x - mu) / sd, with mu and sd
    taken from the training samples, so log q_x(x) = log q_u(u) - sum log sd.
    Draws are u = f^{-1}(z) with z ~ N(0, I) from the sampler's generator.
    Both densities in the acceptance ratio are evaluated by the same forward
    pass, so q is one deterministic function of x.
    """

    def __init__(self, dim: int, n_layers: int = 8, hidden: int = 128, max_batch: int = 65536, seed: int = 0,
                 flow=None):
        from . import mbh
        self.dim = dim
        self.flow = flow if flow is not None else mbh.Flow(dim, n_layers, hidden, max_batch, seed=seed)
        self.mu = np.zeros(dim)
        self.sd = np.ones(dim)
        self.losses = []
        self.train_seconds = 0.0

    def fit(self, x: np.ndarray, steps: int = 400, lr: float = 2e-3, batch: int = 4096, seed: int = 0,
            lr_final: float = None):
        """Adam on minibatches of the samples x [N][dim], the learning rate
        decaying geometrically from lr to lr_final (default lr / 20); returns
        the losses."""
        import torch
        t0 = time.perf_counter()
        x = np.asarray(x, dtype=np.float64).reshape(-1, self.dim)
        self.mu = x.mean(axis=0)
        self.sd = x.std(axis=0) + 1e-12
        u = torch.as_tensor(((x - self.mu) / self.sd).astype(np.float32), device="cuda")
        rng = np.random.default_rng(seed)
        batch = min(batch, len(x), self.flow.max_batch)
        lr_final = lr / 20 if lr_final is None else lr_final
        decay = (lr_final / lr) ** (1.0 / max(steps - 1, 1))
        shift = float(np.sum(np.log(self.sd)))
        for i in range(steps):
            idx = torch.as_tensor(rng.integers(0, len(x), batch), device="cuda")
            loss, _ = self.flow.loss_grad(u.index_select(0, idx), want_grad=False)
            self.flow.adam(lr * decay ** i)
            self.losses.append(loss + shift)
        torch.cuda.synchronize()
        self.train_seconds += time.perf_counter() - t0
        return self.losses

    def propose(self, x_old: np.ndarray, rng: np.random.Generator):
        """n = len(x_old) draws x' ~ q with log q(x') and log q(x_old), in one
        host-to-device copy, an inverse and a forward pass, and one copy back."""
        import torch
        n = len(x_old)
        z = rng.standard_normal((n, self.dim)).astype(np.float32)
        u_old = ((np.asarray(x_old) - self.mu) / self.sd).astype(np.float32)
        dev = torch.as_tensor(np.concatenate([z, u_old]), device="cuda")
        u_new, _ = self.flow.inverse(dev[:n])
        _, lq = self.flow.forward(torch.cat([u_new, dev[n:]]))
        out = torch.cat([u_new.reshape(-1), lq]).cpu().numpy().astype(np.float64)
        u = out[:n * self.dim].reshape(n, self.dim)
        lq = out[n * self.dim:] - float(np.sum(np.log(self.sd)))
        return self.mu + self.sd * u, lq[:n], lq[n:]

    def logq(self, x: np.ndarray) -> np.ndarray:
        u = (np.atleast_2d(x) - self.mu) / self.sd
        _, lq = self.flow.forward(u.astype(np.float32))
        return lq.cpu().numpy().astype(np.float64) - float(np.sum(np.log(self.sd)))

    def sample(self, n: int, rng: np.random.Generator):
        z = rng.standard_normal((n, self.dim)).astype(np.float32)
        u, _ = self.flow.inverse(z)
        x = self.mu + self.sd * u.cpu().numpy().astype(np.float64)
        return x, self.logq(x)


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


# ---------------------------------------------------------------------------
# ESS per second: stretch only against stretch + learned proposal
# ---------------------------------------------------------------------------
def _run_for(smp: PTSampler, seconds: float, chain: list, t_start: float, say=None, every: float = 30.0):
    last = time.perf_counter()
    while time.perf_counter() - t_start < seconds:
        smp.step()
        chain.append(smp.state.x[0].copy())
        if say is not None and time.perf_counter() - last > every:
            last = time.perf_counter()
            say("progress", {"steps": len(chain), "wall_s": round(last - t_start, 1)})


def _arm_report(smp: PTSampler, chain: np.ndarray, wall: float, burn: int):
    post = chain[burn:]
    n_eff, tau, taus = ess(post) if len(post) >= 8 else (0.0, float("inf"), None)
    st = smp.state
    return {
        "steps": int(len(chain)), "burn_in_steps": int(burn), "wall_s": round(wall, 2),
        "like_s": round(smp.like_seconds, 2), "tau": round(float(tau), 2), "ess": round(float(n_eff), 1),
        "ess_per_s": round(float(n_eff) / wall, 3), "chain_over_50_tau": bool(len(post) > 50 * tau),
        "acceptance_per_rung": [round(float(a) / max(1, p), 4) for a, p in zip(st.accepted, st.proposed)],
        "swap_rate": [round(float(a) / max(1, p), 4) for a, p in zip(st.swaps_accepted, st.swaps_proposed)],
        "flow_acceptance": (round(st.flow_accepted / st.flow_proposed, 4) if st.flow_proposed else None),
    }


def ess_comparison(loglike: Callable, logprior: Callable, x0: np.ndarray, betas, seconds: float,
                   seeds=(5, 55), a: float = 1.15, p_flow: float = 0.5, burn_frac: float = 0.3,
                   max_train: int = 200000, flow_kwargs=None, fit_kwargs=None, log=None):
    """Stretch-move PT against stretch + flow PT on the same target, from the
    same start x0[T][W][D], each with the same wall budget 'seconds'.

    Both arms drop their first burn_frac of the budget as burn-in; the flow
    arm trains its proposal on the (thinned) T = 1 samples of that stretch-only
    burn-in, and the training time is charged to it.  ESS (Sec. III.C) counts
    only the post-burn-in T = 1 chain; ESS/s divides by the arm's whole wall
    time.  Accuracy: per-parameter means of the two arms agree within 3
    combined Monte Carlo standard errors, and standard deviations within 5 %.
    """
    say = log or (lambda *_: None)
    dim = x0.shape[-1]
    nw = x0.shape[1]
    out = {}
    # arm 1: stretch only
    smp = PTSampler(loglike, logprior, betas, nw, dim, a=a, seed=seeds[0])
    t0 = time.perf_counter()
    smp.initialize(x0)
    chain: list = []
    _run_for(smp, burn_frac * seconds, chain, t0, say)
    burn = len(chain)
    _run_for(smp, seconds, chain, t0, say)
    ch_plain = np.array(chain)
    out["stretch"] = _arm_report(smp, ch_plain, time.perf_counter() - t0, burn)
    say("stretch", out["stretch"])
    # arm 2: stretch burn-in, flow training, then stretch + flow
    prop = FlowProposal(dim, seed=seeds[1], **(flow_kwargs or {}))
    smp2 = PTSampler(loglike, logprior, betas, nw, dim, a=a, seed=seeds[1], proposal=prop, p_flow=0.0)
    t0 = time.perf_counter()
    smp2.initialize(x0)
    chain = []
    _run_for(smp2, burn_frac * seconds, chain, t0, say)
    burn2 = len(chain)
    train = np.array(chain).reshape(-1, dim)
    if len(train) > max_train:
        train = train[np.linspace(0, len(train) - 1, max_train).astype(int)]
    prop.fit(train, **(fit_kwargs or {}))
    say("flow trained", {"samples": int(len(train)), "train_s": round(prop.train_seconds, 2),
                         "final_loss": round(float(prop.losses[-1]), 4) if prop.losses else None})
    smp2.p_flow = p_flow
    _run_for(smp2, seconds, chain, t0, say)
    ch_flow = np.array(chain)
    out["stretch_flow"] = _arm_report(smp2, ch_flow, time.perf_counter() - t0, burn2)
    out["stretch_flow"]["train_s"] = round(prop.train_seconds, 2)
    out["stretch_flow"]["train_samples"] = int(len(train))
    say("stretch+flow", out["stretch_flow"])
    # equal posterior accuracy between the arms
    a1, a2 = ch_plain[burn:].reshape(-1, dim), ch_flow[burn2:].reshape(-1, dim)
    e1, e2 = max(out["stretch"]["ess"], 1.0), max(out["stretch_flow"]["ess"], 1.0)
    se = np.sqrt(a1.var(0) / e1 + a2.var(0) / e2)
    with np.errstate(divide="ignore", invalid="ignore"):
        zmax = float(np.nanmax(np.abs(a1.mean(0) - a2.mean(0)) / se))
        sd_rel = float(np.nanmax(np.abs(a2.std(0) / a1.std(0) - 1)))
    out["accuracy"] = {"max_mean_diff_in_se": round(zmax, 3), "max_sd_rel_diff": round(sd_rel, 4),
                       "equal": bool(zmax < 3 and sd_rel < 0.05)}
    out["ess_per_s_gain"] = round(out["stretch_flow"]["ess_per_s"] / max(out["stretch"]["ess_per_s"], 1e-12), 3)
    prop.flow.close()
    return out
