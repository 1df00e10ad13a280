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


def adapt_ladder(betas: np.ndarray, swap_frac: np.ndarray, t: int, lag: float, time_scale: float) -> np.ndarray:
    """One step of the adaptive-tempering dynamics (Vousden, Farr and Mandel
    2016, used by the paper through ptemcee, Sec. III.B).

    betas[N] with betas[0] = 1 and betas[-1] = 0 (T_N = infinity);
    swap_frac[N-1] is this step's swap acceptance between rungs k and k+1.
    Interior rung i (1 <= i <= N-2) has the gap g_i = T_i - T_{i-1}; its
    logarithm moves by kappa (swap_frac[i-1] - swap_frac[i]), so a pair that
    swaps more often than the pair above it widens, and the acceptances even
    out.  kappa = (1/time_scale) lag / (t + lag) decays with the step t.
    The gaps are rebuilt from T_0 = 1 upward; the top rung stays at beta = 0.
    """
    betas = np.asarray(betas, dtype=np.float64)
    kappa = lag / (t + lag) / time_scale
    T = 1.0 / betas[:-1]                       # finite rungs T_0 = 1 .. T_{N-2}
    gaps = np.diff(T) * np.exp(kappa * (swap_frac[:-1] - swap_frac[1:]))
    out = betas.copy()
    out[1:-1] = 1.0 / (T[0] + np.cumsum(gaps))
    return out


def ti_evidence(betas, mean_logl):
    """Thermodynamic-integration evidence from parallel-tempered chains:
    ln Z = integral over beta in [0, 1] of <ln L>_beta, where <.>_beta is the
    mean under the tempered posterior proportional to L^beta pi (at beta = 0
    the prior).  The integral is the trapezoid rule over the ladder's betas;
    the error estimate is the difference from the same rule on every other
    rung (the coarser ladder), as is usual for this estimator.

    betas[N] and mean_logl[N] in any order; returns (ln Z, error estimate).
    """
    b = np.asarray(betas, dtype=np.float64)
    m = np.asarray(mean_logl, dtype=np.float64)
    o = np.argsort(b)
    b, m = b[o], m[o]
    if b[0] != 0.0 or b[-1] != 1.0:
        raise ValueError("the ladder must span beta = 0 (T = infinity) to beta = 1")

    def trap(bb, mm):
        return float(np.sum(np.diff(bb) * 0.5 * (mm[1:] + mm[:-1])))

    lnz = trap(b, m)
    keep = np.arange(0, len(b), 2)
    if keep[-1] != len(b) - 1:
        keep = np.append(keep, len(b) - 1)
    coarse = trap(b[keep], m[keep])
    return lnz, abs(lnz - coarse)


def fix_coordinates(fn: Callable, dim: int, fixed: dict) -> Callable:
    """Wrap fn(x[N][dim]) as a function of the free coordinates only: the
    coordinates in 'fixed' (index -> value) are inserted before the call.
    Sec. IV samples Binary 3 with the two spins held at their injected values
    (D = 9 instead of 11); fix_coordinates(loglike, 11, {2: a1, 3: a2}) and the
    same for the prior give that sampler.  The wrapped function has
    .expand(x_free) -> x_full and .free (the free indices)."""
    free = np.array([i for i in range(dim) if i not in fixed], dtype=np.int64)
    idx = np.array(sorted(fixed), dtype=np.int64)
    vals = np.array([fixed[i] for i in sorted(fixed)], dtype=np.float64)

    def expand(xf):
        xf = np.atleast_2d(np.asarray(xf, dtype=np.float64))
        if xf.shape[1] != len(free):
            raise ValueError(f"expected {len(free)} free coordinates, got {xf.shape[1]}")
        x = np.empty((xf.shape[0], dim))
        x[:, free] = xf
        x[:, idx] = vals
        return x

    def wrapped(xf):
        return fn(expand(xf))

    wrapped.expand = expand
    wrapped.free = free
    return wrapped


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


def batch_means_se(chain: np.ndarray, n_batches: int = 20) -> np.ndarray:
    """Standard error of the ensemble mean of chain[N, W, D] per parameter,
    from the spread of the means of n_batches consecutive blocks of steps.
    Unlike the walker-averaged autocorrelation it also sees correlation
    between walkers (an ensemble that drifts or mixes slowly as a whole)."""
    x = np.asarray(chain, dtype=np.float64)
    nb = max(2, min(n_batches, x.shape[0]))
    per = x.shape[0] // nb
    means = x[: nb * per].reshape(nb, per, *x.shape[1:]).mean(axis=(1, 2))   # [nb][D]
    return means.std(axis=0, ddof=1) / math.sqrt(nb)


def ensemble_mean_se(chain: np.ndarray, c_window: float = 5.0) -> np.ndarray:
    """Standard error of the ensemble mean of chain[N, W, D] per parameter,
    from the integrated autocorrelation time of the series of ensemble means
    (the Sokal window above): sqrt(var(m) tau_m / N).  It needs no choice of
    batch length, which biases batch means low when a batch spans only a few
    autocorrelation times of the ensemble as a whole."""
    x = np.asarray(chain, dtype=np.float64)
    m = x.mean(axis=1)                                        # [N][D]
    n = m.shape[0]
    taus = np.array([integrated_time(m[:, d:d + 1], c_window) for d in range(m.shape[1])])
    return m.std(axis=0) * np.sqrt(np.maximum(taus, 1.0) / n)


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
      and .logq(x) -> logq (or .propose(x_old, rng) -> (x, logq, logq_old));
      used with probability p_flow at rungs with beta >= flow_beta_min
      (default: the beta = 1 rungs whose posterior it was trained on).
    adapt: adaptive tempering (Sec. III.B uses ptemcee's; the dynamics are
      those of Vousden, Farr and Mandel 2016): after each round of swaps every
      interior rung i moves so that S_i = ln(T_i - T_{i-1}) changes by
      kappa(t) (A_{i-1,i} - A_{i,i+1}), the difference of this step's swap
      acceptance fractions below and above it, with
      kappa(t) = (1/adapt_time) adapt_lag / (t + adapt_lag).  The coldest
      rung (T = 1) and the top rung stay where they are; the top must be
      T = infinity (beta = 0), as in the paper, so that the ladder stays
      ordered.  Adaptation breaks detailed balance while it acts: switch it
      off (sampler.adapt = False) before keeping samples.
    record_logl: keep ln L of every rung and walker after each step in
      self.logl_history (for the thermodynamic-integration evidence).
    """

    def __init__(self, loglike: Callable, logprior: Callable, betas, n_walkers: int, dim: int,
                 a: float = 1.15, seed: int = 0, proposal=None, p_flow: float = 0.0, flow_beta_min: float = 1.0,
                 adapt: bool = False, adapt_lag: float = 10000.0, adapt_time: float = 100.0,
                 record_logl: bool = False):
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
        self.flow_beta_min = flow_beta_min   # the proposal models the beta = 1 posterior
        if adapt and (self.nt < 3 or self.betas[-1] != 0.0 or self.betas[0] != 1.0):
            raise ValueError("adaptive tempering needs >= 3 rungs from beta = 1 to beta = 0 (T = infinity)")
        self.adapt = adapt
        self.adapt_lag = adapt_lag
        self.adapt_time = adapt_time
        self.record_logl = record_logl
        self.logl_history: list = []
        self.swap_frac = np.zeros(max(self.nt - 1, 0))   # this step's swap acceptance per adjacent pair
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
                use_flow = ((self.rng.random((self.nt, half)) < self.p_flow)
                            & (self.betas[:, None] >= self.flow_beta_min) & (self.betas[:, None] > 0.0))
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
        if self.adapt:
            self.betas = adapt_ladder(self.betas, self.swap_frac, st.step, self.adapt_lag, self.adapt_time)
        if self.record_logl:
            self.logl_history.append(st.logl.copy())
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
            self.swap_frac[i - 1] = acc.mean()

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
        self.betas = z["betas"].copy()        # an adapted ladder resumes where it stood
        self.state = PTState(x=z["x"].copy(), logl=z["logl"].copy(), logp=z["logp"].copy(), step=int(z["step"]),
                             rng_state=rng_state, accepted=z["accepted"].copy(), proposed=z["proposed"].copy(),
                             swaps_accepted=z["swaps_accepted"].copy(), swaps_proposed=z["swaps_proposed"].copy(),
                             flow_accepted=int(fl[0]), flow_proposed=int(fl[1]))
        return self.state


class FlowProposal:
    """Independence proposal: a defensive mixture of the learned affine-coupling
    flow (mbh.Flow) and a broad Gaussian,
        q(x) = (1 - eps) q_flow(x) + eps N(x; m, (infl^2) C),
    with m and C the mean and covariance of the training samples.  The
    Gaussian component bounds pi/q where the flow under-covers the target
    (tails the training chain has not explored), so no walker sticks.

    The flow models standardized coordinates u = (x - mu) / sd, so
    log q_flow(x) = log q_u(u) - sum log sd; it is evaluated as the forward
    pass of float32(u), one deterministic function of x.
    """

    def __init__(self, dim: int, n_layers: int = 8, hidden: int = 128, max_batch: int = 65536, seed: int = 0,
                 flow=None, defensive: float = 0.1, inflate: float = 1.5):
        from . import mbh
        if not 0.0 <= defensive < 1.0:
            raise ValueError("defensive weight must be in [0, 1)")
        self.dim = dim
        self.flow = flow if flow is not None else mbh.Flow(dim, n_layers, hidden, max_batch, seed=seed)
        self.eps = defensive
        self.inflate = inflate
        self.mu = np.zeros(dim)
        self.sd = np.ones(dim)
        self.m = np.zeros(dim)
        self.chol = np.eye(dim)
        self.cinv = np.eye(dim)
        self.gnorm = -0.5 * dim * math.log(2 * math.pi)
        self.losses = []
        self.val_losses = []
        self.train_seconds = 0.0

    def fit(self, x: np.ndarray, steps: int = 600, lr: float = 2e-3, batch: int = 4096, seed: int = 0,
            lr_final: float = None, val_frac: float = 0.2, val_every: int = 25):
        """Adam on minibatches of the samples x [N][dim] (in chain order), the
        learning rate decaying geometrically from lr to lr_final (default
        lr / 20).  The last val_frac of the samples is held out; the
        parameters with the lowest held-out loss are kept."""
        import torch
        t0 = time.perf_counter()
        x = np.asarray(x, dtype=np.float64).reshape(-1, self.dim)
        self.mu = x.mean(axis=0)
        self.sd = x.std(axis=0) + 1e-12
        cov = np.cov(x.T) * self.inflate ** 2 + np.diag((1e-12 * self.sd) ** 2)
        self.m = self.mu.copy()
        self.chol = np.linalg.cholesky(cov)
        self.cinv = np.linalg.inv(cov)
        self.gnorm = -0.5 * (self.dim * math.log(2 * math.pi) + np.linalg.slogdet(cov)[1])
        u_all = torch.as_tensor(((x - self.mu) / self.sd).astype(np.float32), device="cuda")
        nv = int(len(x) * val_frac) if len(x) > 10 else 0
        u, uv = u_all[: len(x) - nv], u_all[len(x) - nv:]
        rng = np.random.default_rng(seed)
        batch = min(batch, len(u), self.flow.max_batch)
        lr_final = lr / 20 if lr_final is None else lr_final
        decay = (lr_final / lr) ** (1.0 / max(steps - 1, 1))
        shift = float(np.sum(np.log(self.sd)))
        best, best_p = float("inf"), None
        for i in range(steps):
            idx = torch.as_tensor(rng.integers(0, len(u), batch), device="cuda")
            loss, _ = self.flow.loss_grad(u.index_select(0, idx), want_grad=False)
            self.flow.adam(lr * decay ** i)
            self.losses.append(loss + shift)
            if nv and (i % val_every == val_every - 1 or i == steps - 1):
                vl = 0.0
                for b0 in range(0, nv, self.flow.max_batch):
                    _, lq = self.flow.forward(uv[b0:b0 + self.flow.max_batch])
                    vl -= float(lq.double().sum())
                vl = vl / nv + shift
                self.val_losses.append(vl)
                if vl < best:
                    best, best_p = vl, self.flow.get_params()
        if best_p is not None:
            self.flow.set_params(best_p)
        torch.cuda.synchronize()
        self.train_seconds += time.perf_counter() - t0
        return self.losses

    def _logq_gauss(self, x):
        d = np.atleast_2d(x) - self.m
        return self.gnorm - 0.5 * np.einsum("ni,ij,nj->n", d, self.cinv, d)

    def _mix(self, lq_flow, x):
        lq_flow = lq_flow - float(np.sum(np.log(self.sd)))
        if self.eps == 0.0:
            return lq_flow
        return np.logaddexp(math.log1p(-self.eps) + lq_flow, math.log(self.eps) + self._logq_gauss(x))

    def logq(self, x: np.ndarray) -> np.ndarray:
        x = np.atleast_2d(x)
        _, lq = self.flow.forward(((x - self.mu) / self.sd).astype(np.float32))
        return self._mix(lq.cpu().numpy().astype(np.float64), x)

    def _buffers(self, rows):
        """Pinned host and device staging for up to 'rows' rows (grown on demand)."""
        import torch
        if getattr(self, "_cap", 0) < rows:
            cap = max(rows, 256)
            f32 = torch.float32
            self._h_in = torch.empty((3 * cap, self.dim), dtype=f32, pin_memory=True)
            self._h_out = torch.empty(cap * self.dim + 3 * cap, dtype=f32, pin_memory=True)
            self._d_in = torch.empty((3 * cap, self.dim), dtype=f32, device="cuda")
            self._d_u = torch.empty((3 * cap, self.dim), dtype=f32, device="cuda")
            self._d_z = torch.empty((3 * cap, self.dim), dtype=f32, device="cuda")
            self._d_lq = torch.empty(3 * cap, dtype=f32, device="cuda")
            self._d_lqi = torch.empty(cap, dtype=f32, device="cuda")
            self._cap = cap

    def propose(self, x_old: np.ndarray, rng: np.random.Generator):
        """len(x_old) draws x' ~ q with log q(x') and log q(x_old).

        Per chunk of rows: one copy of [z; u_gauss; u_old] to the device, an
        inverse pass for the flow draws, one forward pass over the flow draws,
        the Gaussian draws and the old points, and one copy back."""
        import torch
        x_old = np.atleast_2d(x_old)
        n_all = len(x_old)
        gauss = rng.random(n_all) < self.eps
        zn = rng.standard_normal((n_all, self.dim))
        xg = self.m + zn @ self.chol.T
        chunk = max(1, self.flow.max_batch // 3)
        x_new = np.empty((n_all, self.dim))
        lq_f_new = np.empty(n_all)
        lq_f_old = np.empty(n_all)
        for c0 in range(0, n_all, chunk):
            c1 = min(n_all, c0 + chunk)
            n = c1 - c0
            self._buffers(n)
            h = self._h_in.numpy()
            h[:n] = zn[c0:c1]
            h[n:2 * n] = (xg[c0:c1] - self.mu) / self.sd
            h[2 * n:3 * n] = (x_old[c0:c1] - self.mu) / self.sd
            d_in, d_u = self._d_in[:3 * n], self._d_u[:3 * n]
            d_in.copy_(self._h_in[:3 * n], non_blocking=True)
            self.flow.inverse(d_in[:n], out=(d_u[:n], self._d_lqi[:n]))
            d_u[n:].copy_(d_in[n:])
            self.flow.forward(d_u, out=(self._d_z[:3 * n], self._d_lq[:3 * n]))
            ho = self._h_out
            ho[:n * self.dim].view(n, self.dim).copy_(d_u[:n], non_blocking=True)
            ho[n * self.dim:n * self.dim + 3 * n].copy_(self._d_lq[:3 * n], non_blocking=True)
            torch.cuda.current_stream().synchronize()
            o = ho.numpy()
            u_flow = o[:n * self.dim].reshape(n, self.dim).astype(np.float64)
            lq = o[n * self.dim:n * self.dim + 3 * n].astype(np.float64)
            g = gauss[c0:c1]
            u_g = h[n:2 * n].astype(np.float64)
            x_new[c0:c1] = self.mu + self.sd * np.where(g[:, None], u_g, u_flow)
            lq_f_new[c0:c1] = np.where(g, lq[n:2 * n], lq[:n])
            lq_f_old[c0:c1] = lq[2 * n:]
        return x_new, self._mix(lq_f_new, x_new), self._mix(lq_f_old, x_old)

    def sample(self, n: int, rng: np.random.Generator):
        """n draws x ~ q and log q(x)."""
        x, lq, _ = self.propose(np.tile(self.mu, (n, 1)), rng)
        return x, lq


def curvature_covariance(loglike: Callable, x0: np.ndarray, steps: np.ndarray):
    """Covariance (-H)^{-1} from the Hessian H of ln L at x0 by central
    differences with per-coordinate steps, all 1 + 2 D^2 points in one
    batched call:
      H_ii = (f(x + h_i e_i) - 2 f(x) + f(x - h_i e_i)) / h_i^2,
      H_ij = (f(++) - f(+-) - f(-+) + f(--)) / (4 h_i h_j).
    -H is symmetrised and its eigenvalues are held at or above 1e-12 of the
    largest, so the result is a covariance even where ln L is not concave."""
    x0 = np.asarray(x0, dtype=np.float64)
    h = np.asarray(steps, dtype=np.float64)
    d = len(x0)
    pts = [x0]
    for i in range(d):
        for sgn in (1.0, -1.0):
            y = x0.copy()
            y[i] += sgn * h[i]
            pts.append(y)
    pairs = [(i, j) for i in range(d) for j in range(i + 1, d)]
    for i, j in pairs:
        for si, sj in ((1.0, 1.0), (1.0, -1.0), (-1.0, 1.0), (-1.0, -1.0)):
            y = x0.copy()
            y[i] += si * h[i]
            y[j] += sj * h[j]
            pts.append(y)
    f = np.asarray(loglike(np.array(pts)), dtype=np.float64)
    if not np.all(np.isfinite(f)):
        raise ValueError("curvature_covariance: ln L is not finite at some difference points; use smaller steps")
    H = np.zeros((d, d))
    for i in range(d):
        H[i, i] = (f[1 + 2 * i] - 2.0 * f[0] + f[2 + 2 * i]) / (h[i] * h[i])
    base = 1 + 2 * d
    for k, (i, j) in enumerate(pairs):
        fpp, fpm, fmp, fmm = f[base + 4 * k: base + 4 * k + 4]
        H[i, j] = H[j, i] = (fpp - fpm - fmp + fmm) / (4.0 * h[i] * h[j])
    A = -0.5 * (H + H.T)
    lam, V = np.linalg.eigh(A)
    lam = np.maximum(lam, 1e-12 * max(lam.max(), 1e-300))
    return (V / lam) @ V.T


def curvature_start(loglike: Callable, logprior: Callable, x0: np.ndarray, betas, n_walkers: int, seed: int,
                    rel_step: float = 1e-6, refine: int = 1, lo=inputs.PRIOR_LO, hi=inputs.PRIOR_HI):
    """Start positions [T][W][D] for parallel tempering drawn from the Gaussian
    approximation of the posterior at x0: covariance (-H)^{-1} from
    curvature_covariance, widened by the temperature 1/beta on each rung (the
    beta = 0 rung, whose target is the prior, takes four times the largest
    finite temperature), redrawn where the prior is zero; a rung that finds
    too few draws inside the prior narrows by factors of 4.  The first
    Hessian uses steps rel_step |x0_i| (at least rel_step); each refinement
    repeats it with steps of 0.3 of the standard deviations just found.
    Every step stays below a third of the distance from x0 to the edge of the
    box [lo, hi], so all difference points are inside it, and no standard
    deviation exceeds a twentieth of the box's width (a direction the data
    hardly constrain would otherwise start the walkers far outside it)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x0 = np.asarray(x0, dtype=np.float64)
    lo, hi = np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64)
    edge = np.minimum(x0 - lo, hi - x0) / 3.0
    cap = (hi - lo) / 20.0

    def clamp(C):
        s = np.sqrt(np.diag(C))
        f = np.minimum(1.0, cap / np.maximum(s, 1e-300))
        return C * np.outer(f, f)
    steps = np.minimum(rel_step * np.maximum(np.abs(x0), 1.0), edge)
    C = clamp(curvature_covariance(loglike, x0, steps))
    for _ in range(refine):
        C = clamp(curvature_covariance(loglike, x0, np.minimum(0.3 * np.sqrt(np.diag(C)), edge)))
    chol = np.linalg.cholesky(C + 1e-300 * np.eye(len(x0)))
    betas = np.asarray(betas, dtype=np.float64)
    finite = betas[betas > 0]
    t_top = 4.0 / finite.min() if len(finite) else 1.0
    out = np.empty((len(betas), n_walkers, len(x0)))
    for r, b in enumerate(betas):
        t = 1.0 / b if b > 0 else t_top
        filled, tries = 0, 0
        while filled < n_walkers:
            z = rng.standard_normal((n_walkers, len(x0)))
            y = x0 + math.sqrt(t) * z @ chol.T
            ok = np.isfinite(np.asarray(logprior(y)))
            take = y[ok][: n_walkers - filled]
            out[r, filled:filled + len(take)] = take
            filled += len(take)
            tries += 1
            if tries % 20 == 0:
                if t <= 1e-6:
                    raise RuntimeError("curvature_start: too few draws inside the prior")
                t *= 0.25
    return out, C


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


def gpu_loglike_lisa(L, t0):
    """ln L of LISA-frame sampling coordinates (lisaframe.to_sampling_lisa):
    converted to SSB parameters on the host before the waveform, as the
    sampler of Sec. II does, then evaluated through an mbh.Likelihood."""
    from . import lisaframe

    def f(x):
        out = L.loglike(lisaframe.sampling_lisa_to_ssb(np.asarray(x), t0))
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
    # ESS of the ensemble mean from batch means (smallest over parameters):
    # unlike the walker-averaged estimate it counts correlation between walkers
    n_bm = 0.0
    if len(post) >= 40:
        se = batch_means_se(post, 20)
        var = post.reshape(-1, post.shape[-1]).var(axis=0)
        with np.errstate(divide="ignore", invalid="ignore"):
            n_bm = float(np.nanmin(np.where(se > 0, var / se ** 2, np.inf)))
    st = smp.state
    # integrated time of the ensemble mean implied by the batch-means ESS
    tau_bm = float(post.shape[0] * post.shape[1] / n_bm) if n_bm > 0 else float("inf")
    return {
        "steps": int(len(chain)), "burn_in_steps": int(burn), "wall_s": round(wall, 2),
        "ensemble_tau_batch_means": round(tau_bm, 2), "chain_over_50_ensemble_tau": bool(len(post) > 50 * tau_bm),
        "like_s": round(smp.like_seconds, 2), "tau": round(float(tau), 2), "ess": round(float(n_eff), 1),
        "ess_per_s": round(float(n_eff) / wall, 3), "chain_over_50_tau": bool(len(post) > 50 * tau),
        "ess_batch_means": round(n_bm, 1), "ess_batch_means_per_s": round(n_bm / wall, 3),
        "acceptance_per_rung": [round(float(a) / max(1, p), 4) for a, p in zip(st.accepted, st.proposed)],
        "swap_rate": [round(float(a) / max(1, p), 4) for a, p in zip(st.swaps_accepted, st.swaps_proposed)],
        "flow_acceptance": (round(st.flow_accepted / st.flow_proposed, 4) if st.flow_proposed else None),
    }


def ess_comparison(loglike: Callable, logprior: Callable, x0: np.ndarray, betas, seconds: float,
                   burn_seconds: float, seeds=(5, 55), a: float = 1.15, p_flow: float = 0.8,
                   max_train: int = 200000, flow_kwargs=None, fit_kwargs=None, log=None, keep_chains=False):
    """Stretch-move PT against stretch + flow PT on the same target.

    One stretch-only burn-in of burn_seconds from x0[T][W][D] is shared and
    charged to neither arm.  From its final state the plain arm keeps
    running, and the flow arm trains its proposal on the T = 1 samples of
    the burn-in's second half (thinned to at most max_train) and then runs
    with independence proposals at probability p_flow on the T = 1 rung;
    each arm gets the same wall budget
    'seconds', the flow arm's training included.  ESS (Sec. III.C) counts
    the arm's T = 1 chain; ESS/s divides by the arm's wall time.  Accuracy:
    per-parameter means of the two arms agree within 3 combined Monte Carlo
    standard errors of the ensemble means (each arm's the larger of its
    batch means and its autocorrelation estimate), and standard deviations
    within 5 %.  Also reported: the mean differences in walker-averaged and
    in batch-means standard errors (the latter see correlation between
    walkers) and each arm's first half against its second half (a drift
    check).  keep_chains adds both arms' T = 1 chains to the result under
    'chains'.
    """
    say = log or (lambda *_: None)
    dim = x0.shape[-1]
    nw = x0.shape[1]
    out = {}
    base = PTSampler(loglike, logprior, betas, nw, dim, a=a, seed=seeds[0])
    t0 = time.perf_counter()
    base.initialize(x0)
    warm: list = []
    _run_for(base, burn_seconds, warm, t0, say)
    start = base.state.x.copy()
    out["burn_in"] = {"steps": len(warm), "wall_s": round(time.perf_counter() - t0, 2)}
    say("burn-in", out["burn_in"])
    # arm 1: stretch only, continuing the burn-in
    base.state.accepted[:] = 0
    base.state.proposed[:] = 0
    base.state.swaps_accepted[:] = 0
    base.state.swaps_proposed[:] = 0
    t0 = time.perf_counter()
    chain: list = []
    _run_for(base, seconds, chain, t0, say)
    ch_plain = np.array(chain)
    out["stretch"] = _arm_report(base, ch_plain, time.perf_counter() - t0, 0)
    say("stretch", out["stretch"])
    # arm 2: train on the burn-in, then stretch + flow from the same state
    t0 = time.perf_counter()
    settled = np.array(warm[len(warm) // 2:])        # the second half of the burn-in
    keep = np.linspace(0, len(settled) - 1, max(1, min(len(settled), max_train // nw))).astype(int)
    train = settled[keep].reshape(-1, dim)
    prop = FlowProposal(dim, seed=seeds[1], **(flow_kwargs or {}))
    prop.fit(train, **(fit_kwargs or {}))
    say("flow trained", {"samples": int(len(train)), "train_s": round(prop.train_seconds, 2),
                         "best_held_out_loss": round(min(prop.val_losses), 4) if prop.val_losses else None})
    smp = PTSampler(loglike, logprior, betas, nw, dim, a=a, seed=seeds[1], proposal=prop, p_flow=p_flow)
    smp.initialize(start)
    chain = []
    _run_for(smp, seconds, chain, t0, say)
    ch_flow = np.array(chain)
    out["stretch_flow"] = _arm_report(smp, ch_flow, time.perf_counter() - t0, 0)
    out["stretch_flow"]["train_s"] = round(prop.train_seconds, 2)
    out["stretch_flow"]["train_samples"] = int(len(train))
    say("stretch+flow", out["stretch_flow"])
    a1, a2 = ch_plain.reshape(-1, dim), ch_flow.reshape(-1, dim)
    e1, e2 = max(out["stretch"]["ess"], 1.0), max(out["stretch_flow"]["ess"], 1.0)
    se = np.sqrt(a1.var(0) / e1 + a2.var(0) / e2)
    se_bm = np.sqrt(batch_means_se(ch_plain) ** 2 + batch_means_se(ch_flow) ** 2)
    # each arm's standard error of the ensemble mean: the larger of its
    # batch means and its autocorrelation estimate (batches a few ensemble
    # autocorrelation times long bias the batch means low)
    se_hi = np.sqrt(np.maximum(batch_means_se(ch_plain), ensemble_mean_se(ch_plain)) ** 2 +
                    np.maximum(batch_means_se(ch_flow), ensemble_mean_se(ch_flow)) ** 2)
    h = len(ch_plain) // 2
    se_drift = np.sqrt(batch_means_se(ch_plain[:h], 10) ** 2 + batch_means_se(ch_plain[h:], 10) ** 2)
    hf = len(ch_flow) // 2
    se_drift_f = np.sqrt(batch_means_se(ch_flow[:hf], 10) ** 2 + batch_means_se(ch_flow[hf:], 10) ** 2)
    with np.errstate(divide="ignore", invalid="ignore"):
        z = np.abs(a1.mean(0) - a2.mean(0)) / se
        z_bm = np.abs(a1.mean(0) - a2.mean(0)) / se_bm
        z_hi = np.abs(a1.mean(0) - a2.mean(0)) / se_hi
        z_drift = np.abs(ch_plain[:h].reshape(-1, dim).mean(0) - ch_plain[h:].reshape(-1, dim).mean(0)) / se_drift
        z_drift_f = np.abs(ch_flow[:hf].reshape(-1, dim).mean(0) - ch_flow[hf:].reshape(-1, dim).mean(0)) / se_drift_f
        zmax = float(np.nanmax(z))
        sd_rel = float(np.nanmax(np.abs(a2.std(0) / a1.std(0) - 1)))
    zmax_bm = float(np.nanmax(z_bm))
    zmax_hi = float(np.nanmax(z_hi))
    # equal accuracy is judged on standard errors of the ensemble mean (the
    # larger of batch means and autocorrelation): the walker-averaged
    # estimate misses correlation between walkers and understates the error
    # of an ensemble's mean
    out["accuracy"] = {"max_mean_diff_in_se": round(zmax, 3), "max_sd_rel_diff": round(sd_rel, 4),
                       # the comparison needs runs longer than 50 times the
                       # integrated time, here that of the ensemble mean
                       "runs_over_50_ensemble_tau": bool(out["stretch"]["chain_over_50_ensemble_tau"] and
                                                         out["stretch_flow"]["chain_over_50_ensemble_tau"]),
                       "max_mean_diff_in_batch_means_se": round(zmax_bm, 3),
                       "max_mean_diff_in_ensemble_se": round(zmax_hi, 3),
                       "equal": bool(zmax_hi < 3 and sd_rel < 0.05),
                       "mean_diff_in_se": [round(float(v), 2) for v in z],
                       "mean_diff_in_batch_means_se": [round(float(v), 2) for v in z_bm],
                       "stretch_arm_half_vs_half_in_batch_means_se": [round(float(v), 2) for v in z_drift],
                       "flow_arm_half_vs_half_in_batch_means_se": [round(float(v), 2) for v in z_drift_f]}
    if keep_chains:
        out["chains"] = (ch_plain, ch_flow)
    out["ess_per_s_gain"] = round(out["stretch_flow"]["ess_per_s"] / max(out["stretch"]["ess_per_s"], 1e-12), 3)
    out["ess_per_s_gain_batch_means"] = round(out["stretch_flow"]["ess_batch_means_per_s"] /
                                              max(out["stretch"]["ess_batch_means_per_s"], 1e-12), 3)
    prop.flow.close()
    return out
