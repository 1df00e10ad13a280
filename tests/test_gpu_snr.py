"""GPU parity of the per-mode SNR decomposition (Sec. IV, Table III): the
optimal SNR rho^2 = sum_c <h|h>_c of every mode subset, and the
matched-filter SNR in noise, from libmbh's dense kernel against the FP64
oracle on the same inputs.  Tolerance: rho^2 to 1e-10 relative; the
matched-filter SNR to 1e-10 of sqrt(<d|d>)."""
import math

import numpy as np
import pytest

from paper_2005_01827_amd import inputs

pytestmark = pytest.mark.gpu

RTOL = 1e-10


def _oracle_subsets(oracle, th, grid, data, psd, ns, t0):
    res = {}
    for key, modes in [("all", inputs.MODES_ALL)] + [(lm, [lm]) for lm in inputs.MODES_ALL]:
        res[key] = oracle.loglike(np.atleast_2d(th), grid, data, psd, modes, ns, t0)
    return res


def test_mode_snr_small_grid_in_noise(oracle):
    """Each subset injected alone (the oracle's template) into one noise
    realisation: rho and the matched-filter SNR against the oracle, and the
    matched-filter SNR of the source itself within 5 of rho."""
    from paper_2005_01827_amd import snr
    w = inputs.small_config(1)
    g = w.grid
    psd = inputs.psd_aet(g.freqs)
    noise = inputs.noise(g, psd, 31)
    subsets = [("all", inputs.MODES_ALL)] + [(lm, [lm]) for lm in inputs.MODES_ALL]
    data = {key: oracle.template(w.injection, g, modes, w.ns, w.t0) + noise for key, modes in subsets}
    N = 8
    th = np.repeat(w.injection[None], N, axis=0)
    th[:, 5] = (w.injection[5] + 2 * math.pi * np.arange(N) / N) % (2 * math.pi)   # walker 0 = injection
    print(f"case: mode SNRs, small grid, {N} walkers in phi_ref, each subset alone in noise seed 31", flush=True)
    with snr.ModeSNR(g, psd, w.modes, w.ns, w.t0, data=data, max_batch=N) as S:
        got = S(th)
    for key, modes in subsets:
        o = oracle.loglike(th, g, data[key], psd, modes, w.ns, w.t0)
        rho, mf = got[key]
        hh = o[:, 4:7].sum(axis=1)
        mf_o = o[:, 1:4].sum(axis=1) / np.sqrt(hh)
        dd = float(np.sum(4 * g.df * np.abs(data[key]) ** 2 / psd))
        assert np.all(np.abs(rho ** 2 / hh - 1) < RTOL), key
        assert np.all(np.abs(mf - mf_o) < RTOL * math.sqrt(dd)), key
        assert abs(mf[0] - rho[0]) < 5.0, (key, mf[0], rho[0])
        if key != "all":
            # one mode alone: rho does not depend on phi_ref
            assert np.max(np.abs(rho / rho[0] - 1)) < 1e-12, key


def test_mode_snr_table2_binaries_full_grid(oracle):
    from paper_2005_01827_amd import snr
    w = inputs.year_grid(1)
    g = w.grid
    psd = inputs.psd_aet(g.freqs)
    bins = (1, 4, 5, 6, 7)
    th = np.stack([inputs.table2_binaries()[b] for b in bins])
    print(f"case: mode SNRs of Table II binaries {bins}, 2^25-s grid, zero noise", flush=True)
    got = snr.mode_snrs(g, psd, th, w.modes, w.ns, w.t0)
    zero = np.zeros((3, g.n), complex)
    ref = _oracle_subsets(oracle, th, g, zero, psd, w.ns, w.t0)
    for key, o in ref.items():
        rho, mf = got[key]
        assert mf is None
        hh = o[:, 4:7].sum(axis=1)
        err = np.abs(rho ** 2 / hh - 1)
        print(f"[{key}] rho {np.round(rho, 1)} max rel err {err.max():.2e}", flush=True)
        assert np.all(err < RTOL), key
