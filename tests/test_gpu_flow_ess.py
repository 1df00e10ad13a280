"""ESS per second of stretch + learned proposal against stretch only.

Target: an 11-D curved ('banana') density, which an affine-invariant stretch
move mixes slowly along its curved ridge.  Both runs start from the same
exact draws, use the same seeds and the same number of likelihood
evaluations; the flow run spends its first sixth on stretch moves whose
samples train the flow (the training time is charged to the flow run).
ESS uses the Sokal-window integrated time of Sec. III.C.  Both runs must
reach the same posterior accuracy: every mean within 4 Monte Carlo standard
errors and every standard deviation within 5 % of the exact values.
"""
import math
import time

import numpy as np
import pytest

from paper_2005_01827_amd import inputs
from paper_2005_01827_amd import sampler as S

pytestmark = pytest.mark.gpu

DIM, NW, B, SX = 11, 64, 0.6, 2.0
STEPS = 3600


def _loglike(x):
    x = np.atleast_2d(x)
    r1 = x[:, 1] - B * (x[:, 0] ** 2 - SX * SX)
    return -0.5 * ((x[:, 0] / SX) ** 2 + r1 * r1 + np.sum(x[:, 2:] ** 2, axis=1))


def _exact_moments():
    mean = np.zeros(DIM)
    sd = np.ones(DIM)
    sd[0] = SX
    sd[1] = math.sqrt(2 * B * B * SX ** 4 + 1)          # Var[b (x0^2 - sx^2)] + 1
    return mean, sd


def _accuracy(chain, n_eff):
    flat = chain.reshape(-1, DIM)
    mean, sd = _exact_moments()
    z = np.abs(flat.mean(0) - mean) / (sd / math.sqrt(n_eff))
    rel = np.abs(flat.std(0) / sd - 1)
    return z.max(), rel.max()


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_flow_raises_ess_per_second(gpu):
    flat = lambda x: np.zeros(len(np.atleast_2d(x)))
    x0 = inputs.banana(NW, DIM, 5, B, SX)[None]

    t = time.perf_counter()
    base = S.PTSampler(_loglike, flat, [1.0], NW, DIM, a=2.0, seed=5)
    base.initialize(x0)
    ch_b = base.run(STEPS)
    wall_b = time.perf_counter() - t
    ess_b, tau_b, _ = S.ess(ch_b)

    t = time.perf_counter()
    prop = S.FlowProposal(DIM, max_batch=8192, seed=55)
    fl = S.PTSampler(_loglike, flat, [1.0], NW, DIM, a=2.0, seed=5, proposal=prop, p_flow=0.0)
    fl.initialize(x0)
    warm = fl.run(STEPS // 6)
    prop.fit(warm.reshape(-1, DIM), steps=300, lr=2e-3, batch=4096, seed=55)
    fl.p_flow = 0.5
    ch_f = fl.run(STEPS - STEPS // 6)
    wall_f = time.perf_counter() - t
    ess_f, tau_f, _ = S.ess(ch_f)

    acc_f = fl.state.flow_accepted / max(1, fl.state.flow_proposed)
    zb, rb = _accuracy(ch_b, ess_b)
    zf, rf = _accuracy(ch_f, ess_f)
    print(f"stretch only: tau {tau_b:.1f} ESS {ess_b:.0f} in {wall_b:.2f} s -> {ess_b / wall_b:.0f} ESS/s; "
          f"accuracy z {zb:.2f}, sd {rb:.3f}")
    print(f"stretch+flow: tau {tau_f:.1f} ESS {ess_f:.0f} in {wall_f:.2f} s (training {prop.train_seconds:.2f} s) "
          f"-> {ess_f / wall_f:.0f} ESS/s; flow acceptance {acc_f:.2f}; accuracy z {zf:.2f}, sd {rf:.3f}")
    # Both runs longer than 50 tau (Sec. III.C) and equally accurate.
    assert len(ch_b) > 50 * tau_b and len(ch_f) > 50 * tau_f
    assert zf < 4 and rf < 0.05
    assert zb < 4 and rb < 0.05
    # Per likelihood evaluation and per second.
    assert ess_f / (STEPS * NW) > 5 * ess_b / (STEPS * NW)
    assert ess_f / wall_f > 2 * ess_b / wall_b
