"""Per-mode signal-to-noise decomposition on the batched likelihood.

Sec. IV (Table III) reports the SNR of each test binary with all harmonic
modes and with each mode in isolation.  Here the optimal SNR of walker b is

    rho_b = sqrt( sum_{c in A,E,T} <h_b | h_b>_c )          (Sec. II, Eq. innerprod)

for the template built from a mode subset, and, when data d are given, the
matched-filter SNR  sum_c Re<d|h>_c / rho_b.  In zero noise with d = h the two
are equal; when the data hold exactly that subset's template plus noise, the
matched-filter SNR scatters about rho with unit variance.  Table III computes
each mode in isolation; isolated_in_noise() is the same decomposition in noise,
with each subset's injection alone in one shared noise realisation.

Every inner product runs in the dense kernel of libmbh (mbh_interp_and_inner);
this module only opens one context per mode subset and divides.  Modes are
fixed per context (the mode list is part of the context descriptor), so a
decomposition over the six modes opens seven contexts that share nothing but
the host data.
"""
from __future__ import annotations

import numpy as np

from . import inputs, mbh


class ModeSNR:
    """Contexts for the full mode set and for each mode alone.

    grid, psd, modes, n_sparse, t0 as for mbh.Likelihood.  data is None
    (zero data: the matched-filter SNR is not reported), one complex [3][n]
    array shared by every subset, or a dict keyed "all" and (l, m) with one
    array per subset.
    """

    def __init__(self, grid, psd, modes=inputs.MODES_ALL, n_sparse=256, t0=0.0, data=None, max_batch=64,
                 precision=mbh.MBH_FP64):
        self.modes = tuple(tuple(m) for m in modes)
        self.have_data = data is not None
        self.subsets = [("all", self.modes)] + [(m, (m,)) for m in self.modes]
        self.ctx = {}
        try:
            for key, sub in self.subsets:
                if data is None:
                    d = np.zeros((3, grid.n), dtype=np.complex128)
                elif isinstance(data, dict):
                    d = data[key]
                else:
                    d = data
                self.ctx[key] = mbh.Likelihood(grid, d, psd, sub, n_sparse, t0, precision=precision,
                                               max_batch=max_batch)
        except BaseException:
            self.close()
            raise

    def __call__(self, params) -> dict:
        """{key: (rho [B], rho_mf [B] or None)} for key = "all" and each (l, m).

        Walkers the likelihood rejects (outside the physical range) get NaN.
        """
        out = {}
        for key, _ in self.subsets:
            o = self.ctx[key].stages(params).cpu().numpy()
            hh = o[:, 4:7].sum(axis=1)
            dh = o[:, 1:4].sum(axis=1)
            bad = ~np.isfinite(o[:, 0])
            rho = np.sqrt(np.where(bad, np.nan, hh))
            mf = None
            if self.have_data:
                with np.errstate(invalid="ignore", divide="ignore"):
                    mf = np.where(bad | (hh <= 0.0), np.nan, dh / rho)
            out[key] = (rho, mf)
        return out

    def close(self):
        for c in self.ctx.values():
            c.close()
        self.ctx = {}

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def mode_snrs(grid, psd, params, modes=inputs.MODES_ALL, n_sparse=256, t0=0.0, data=None) -> dict:
    """One-shot form of ModeSNR: opens the contexts, evaluates, closes."""
    B = np.atleast_2d(np.asarray(params)).shape[0]
    with ModeSNR(grid, psd, modes, n_sparse, t0, data, max_batch=max(B, 1)) as s:
        return s(params)



def isolated_in_noise(grid, psd, theta, noise, modes=inputs.MODES_ALL, n_sparse=256, t0=0.0) -> dict:
    """Table III's decomposition in noise for one source theta [11]: for each
    subset ("all" and every mode alone) the data are that subset's template
    of theta plus the same noise [3][n]; returns {key: (rho, rho_mf)} as
    ModeSNR does, each a length-1 array.  The templates come from libmbh's
    template entry point."""
    theta = np.asarray(theta, dtype=np.float64).reshape(1, 11)
    with ModeSNR(grid, psd, modes, n_sparse, t0, max_batch=1) as s0:
        data = {key: s0.ctx[key].template(theta).cpu().numpy() + noise for key, _ in s0.subsets}
    with ModeSNR(grid, psd, modes, n_sparse, t0, data=data, max_batch=1) as s:
        return s(theta)
