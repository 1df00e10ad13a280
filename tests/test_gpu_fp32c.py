"""GPU parity of the FP32C dense stage (FP64 phase, FP32 template, residual
form of Eq. NLL with the whitened data as an FP32 pair and float-float
residual sums) against the FP64 oracle.

Error model (written from the kernel's arithmetic, before measuring).  The
only FP32 quantity in ln L is the template: the data enter exactly (about 48
bits), the residual d - h is formed exactly by TwoSum, its square by an FMA
TwoProd, and the sums are float-float, so the summation error is of order
u^2 sum |r|^2 (u = 2^-24), below 1e-7 here.  A template error dh_k moves ln L
by Re<d - h, dh> (first order).  Per mode-bin the FP32 chain has about 15
roundings relative to |T_lm A_lm| (the offset cast, the amplitude cubic with
its coefficient rounding, the quarter-turn remainder and the sine/cosine
polynomials, the product A e^{i phi}, the response cubic); the complex
multiply-accumulate over six modes adds 12 roundings relative to H_k =
sum_lm |T_lm A_lm| and the whitening by sqrt(w) in FP32 two more: 29 in all.
Taken as independent, each uniform within +-u of its operand, they give a
relative template error of rms sigma_rel = u sqrt(29/3) of H_k, independent
from bin to bin, so that ln L carries an error of rms

    sigma_w = sigma_rel * sqrt( sum_k |r~_k|^2 H~_k^2 / 2 ),

with r~ = (d - h) sqrt(w) and H~ = H sqrt(w).  Near the data (r ~ noise,
|r~_k|^2 ~ 2) that is sigma_rel times about rho_H: a floor of one FP32
rounding times the SNR, scaled by the number of roundings (about 1.9e-5 at
SNR 100, 1.9e-4 at SNR 1000).  The test allows 6 sigma_w, plus the FP64 parity tolerance
1e-10 max(|ln L|, 1) of the sparse stage and phase, plus 1e-6 for the
float-float sums.  sigma_w is computed per walker from the oracle's
per-mode templates.
"""
import math
import os

import numpy as np
import pytest

from paper_2005_01827_amd import inputs

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
N_ROUND = 29
SIG_REL = U32 * math.sqrt(N_ROUND / 3.0)
TAIL = 6.0


def model_sigma(oracle, walkers, grid, data, psd, modes, ns, t0):
    """sigma_w of the error model for each walker (0 for an invalid one)."""
    w = 4.0 * grid.df / psd
    out = np.zeros(len(walkers))
    for i, th in enumerate(walkers):
        hm = [oracle.template(th, grid, [m], ns, t0) for m in modes]
        h = np.sum(hm, axis=0)
        H = np.sum([np.abs(x) for x in hm], axis=0)
        out[i] = SIG_REL * math.sqrt(0.5 * float(np.sum(np.abs(data - h) ** 2 * w * H * H * w)))
    return out


def bound(sig, lnl_ref):
    return TAIL * sig + 1e-10 * np.maximum(np.abs(lnl_ref), 1.0) + 1e-6


def _scaled(w, snr, oracle, psd):
    """Injection and walkers with D_L scaled so that the injection has the
    given optimal SNR (the template scales as 1/D_L exactly)."""
    g = w.grid
    h = oracle.template(w.injection, g, w.modes, w.ns, w.t0)
    rho0 = math.sqrt(float(np.sum(np.abs(h) ** 2 * 4.0 * g.df / psd)))
    f = rho0 / snr
    inj = w.injection.copy()
    inj[4] *= f
    return inj, h / f


@pytest.mark.parametrize("snr", [100.0, 1000.0])
def test_fp32c_small_grid_error_model(oracle, snr):
    """Walkers on the injection, in a tight ball about it (the sampler's
    regime: residual ~ noise) and in the 1e-3 ball, at SNR 100 and 1000."""
    import torch
    from paper_2005_01827_amd import mbh
    print(f"case: FP32C small grid, SNR {snr}", flush=True)
    w = inputs.small_config(8, seed=7)
    g = w.grid
    psd = inputs.psd_aet(g.freqs)
    inj, h = _scaled(w, snr, oracle, psd)
    d = h + inputs.noise(g, psd, 77)
    walkers = np.concatenate([inj[None], inputs.ball(inj, 5, 1e-6, 41), inputs.ball(inj, 6, 1e-3, 42)])
    L = mbh.Likelihood(g, d, psd, w.modes, w.ns, w.t0, precision=mbh.MBH_FP32C, max_batch=16)
    try:
        out = L.stages(walkers).cpu().numpy()
        lnl = L.loglike(walkers).cpu().numpy()
        # one walker alone (fused sparse kernel, the one-walker dense
        # kernel) gives its batched value bit for bit
        ones = np.array([L.loglike(walkers[i:i + 1]).cpu().numpy()[0] for i in (0, 6, 11)])
        torch.cuda.synchronize()
    finally:
        L.close()
    assert np.array_equal(ones, lnl[[0, 6, 11]]), (ones, lnl[[0, 6, 11]])
    ref = oracle.loglike(walkers, g, d, psd, w.modes, w.ns, w.t0)
    sig = model_sigma(oracle, walkers, g, d, psd, w.modes, w.ns, w.t0)
    err = np.abs(out[:, 0] - ref[:, 0])
    b = bound(sig, ref[:, 0])
    print(f"[fp32c-small snr={snr:.0f}] |dlnL| max {err.max():.3e}  err/sigma max {np.max(err / sig):.2f}  "
          f"sigma {sig.min():.2e}..{sig.max():.2e}", flush=True)
    # the graph-launched residual-only kernel and the inner-product kernel
    # form the same residual sums in the same order
    assert np.array_equal(lnl, out[:, 0])
    assert np.all(err <= b), (err, b)
    hh = ref[:, 4:7].sum(1)
    assert np.all(np.abs(out[:, 4:7].sum(1) - hh) <= 1e-5 * hh)


def test_fp32c_noiseless_injection_is_small(oracle):
    """Zero-noise data equal to the oracle template: ln L(FP64) ~ 0, and the
    FP32C error is the template error alone."""
    import torch
    from paper_2005_01827_amd import mbh
    print("case: FP32C noiseless injection, small grid", flush=True)
    w = inputs.small_config(2, seed=7)
    g = w.grid
    psd = inputs.psd_aet(g.freqs)
    inj, h = _scaled(w, 300.0, oracle, psd)
    L = mbh.Likelihood(g, h, psd, w.modes, w.ns, w.t0, precision=mbh.MBH_FP32C, max_batch=2)
    try:
        got = L.loglike(inj[None]).cpu().numpy()
        torch.cuda.synchronize()
    finally:
        L.close()
    # with r = 0 the first-order term vanishes: ln L = -<dh, dh>/2, of order
    # (sigma_rel rho)^2
    rho = 300.0
    print(f"[fp32c-noiseless] lnL = {got[0]:.3e}", flush=True)
    assert got[0] <= 0.0
    assert abs(got[0]) <= (TAIL * SIG_REL * 1.5 * rho) ** 2 + 1e-6


@pytest.mark.slow
def test_fp32c_tobs25_sampled(oracle):
    """The 1024-walker batch on the T_obs = 2^25 s grid (SNR ~1760 at the
    injection), with checked walkers that include the shortest and longest
    union bands."""
    import torch
    from paper_2005_01827_amd import mbh
    print("case: FP32C, T_obs=2^25 grid, 1024 walkers, 8 checked", flush=True)
    w = inputs.year_grid(1024)
    g = w.grid
    psd = inputs.psd_aet(g.freqs)
    d = oracle.template(w.injection, g, w.modes, w.ns, w.t0) + inputs.noise(g, psd, 2002)
    L = mbh.Likelihood(g, d, psd, w.modes, w.ns, w.t0, precision=mbh.MBH_FP32C, max_batch=1024)
    try:
        got = L.loglike(w.walkers).cpu().numpy()
        torch.cuda.synchronize()
        span = np.array([int(b[b[:, 0] == 1, 2].max() - b[b[:, 0] == 1, 1].min())
                         for b in (L.get_sparse(i)["band"] for i in range(1024))])
    finally:
        L.close()
    idx = np.unique(np.concatenate([[int(np.argmin(span)), int(np.argmax(span))],
                                    np.linspace(0, 1023, 6).astype(int)]))
    nthreads = min(16, os.cpu_count() or 1)
    ref = oracle.loglike(w.walkers[idx], g, d, psd, w.modes, w.ns, w.t0, nthreads=nthreads)
    sig = model_sigma(oracle, w.walkers[idx], g, d, psd, w.modes, w.ns, w.t0)
    err = np.abs(got[idx] - ref[:, 0])
    print(f"[fp32c-tobs25] max |dlnL| = {err.max():.3e}  err/sigma max {np.max(err / sig):.2f}  "
          f"SNR ~ {np.sqrt(ref[:, 4:7].sum(1)).mean():.0f}", flush=True)
    assert np.all(err <= bound(sig, ref[:, 0])), (err, bound(sig, ref[:, 0]))
