"""The paper's sampler settings on the batched MBHB likelihood (Sec. III.B and
Sec. IV): the 10-rung ladder with T_10 = infinity and the finite rungs at
2.04807^k, stretch scale a = 1.15, adaptive tempering, and Binary 3's
fixed-spin sampling (D = 9); the thermodynamic-integration evidence from the
same chains.  Every likelihood call is one batch of all rungs' walkers through
libmbh."""
import numpy as np
import pytest

from paper_2005_01827_amd import inputs
from paper_2005_01827_amd import sampler as S

pytestmark = pytest.mark.gpu


def test_fixed_spin_adaptive_pt_on_mbhb_likelihood(oracle):
    from paper_2005_01827_amd import mbh
    w = inputs.small_config(1)
    g = w.grid
    psd = inputs.psd_aet(g.freqs)
    data = oracle.template(w.injection, g, w.modes, w.ns, w.t0) + inputs.noise(g, psd, 303)
    nt, nw = 10, 32
    L = mbh.Likelihood(g, data, psd, w.modes, w.ns, w.t0, max_batch=nt * nw)
    try:
        x_inj = inputs.to_sampling(w.injection)
        fixed = {2: float(x_inj[2]), 3: float(x_inj[3])}
        ll9 = S.fix_coordinates(S.gpu_loglike(L), 11, fixed)
        lp9 = S.fix_coordinates(S.box_logprior(), 11, fixed)
        free = ll9.free
        rng = np.random.default_rng(304)
        x0 = x_inj[free] + 1e-4 * np.abs(x_inj[free]) * rng.standard_normal((nt, nw, len(free)))
        print("case: 10-rung adaptive PT, D = 9 (spins fixed), small grid, 32 walkers per rung", flush=True)
        smp = S.PTSampler(ll9, lp9, S.ladder(nt), nw, len(free), a=1.15, seed=305, adapt=True, adapt_lag=100,
                          adapt_time=10, record_logl=True)
        smp.initialize(x0)
        smp.run(150)
        smp.adapt = False
        smp.logl_history.clear()
        chain = smp.run(150)
    finally:
        L.close()
    b = smp.betas
    assert b[0] == 1.0 and b[-1] == 0.0 and np.all(np.diff(b) < 0)
    assert not np.array_equal(b, S.ladder(nt))                 # the ladder moved
    full = ll9.expand(chain.reshape(-1, len(free)))
    assert np.all(full[:, 2] == fixed[2]) and np.all(full[:, 3] == fixed[3])
    assert np.all(inputs.in_prior(full))
    acc = smp.state.accepted[0] / smp.state.proposed[0]
    assert 0.02 < acc < 0.95, acc
    hist = np.array(smp.logl_history)                         # [steps][T][W]
    lnz, err = S.ti_evidence(b, hist.mean(axis=(0, 2)))
    print(f"cold acceptance {acc:.3f}; T = {np.round(1 / b[:-1], 2)}; ln Z = {lnz:.1f} +- {err:.1f}; "
          f"max ln L = {hist[:, 0].max():.1f}", flush=True)
    assert np.isfinite(lnz) and lnz < hist[:, 0].max()
    # the cold chain sits at the injection's likelihood scale: -2 ln L of the
    # injection is chi^2 of the noise, about 2 per bin and channel
    assert hist[:, 0].max() > -4 * 3 * g.n
