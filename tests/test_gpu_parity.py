"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
the same seeded inputs.

Tolerance (FP64 path): |lnL_gpu - lnL_oracle| <= 1e-10 max(|lnL|, 1); the
inner products <d|h>_c, <h|h>_c to 1e-10 of sqrt(<h|h>) <d|d>-scale.  Integer
results (band edges, active flags) must match exactly."""
import ctypes
import math
import os

import numpy as np
import pytest

from paper_2005_01827_amd import inputs

pytestmark = pytest.mark.gpu

RTOL = 1e-10


def _lnl_close(g, o):
    g, o = np.asarray(g), np.asarray(o)
    both_inf = np.isneginf(g) & np.isneginf(o)
    ok = both_inf | (np.abs(g - o) <= RTOL * np.maximum(np.abs(o), 1.0))
    return ok


def _report(name, g, o):
    err = np.abs(np.asarray(g) - np.asarray(o)) / np.maximum(np.abs(np.asarray(o)), 1.0)
    err = err[np.isfinite(err)]
    print(f"[{name}] max rel err {err.max() if err.size else 0:.3e}", flush=True)


@pytest.fixture(scope="module")
def small(oracle):
    import torch
    from paper_2005_01827_amd import mbh
    w = inputs.small_config(8, seed=7)
    g = w.grid
    psd = inputs.psd_aet(g.freqs)
    h = oracle.template(w.injection, g, w.modes, w.ns, w.t0)
    d = h + inputs.noise(g, psd, 77)
    L = mbh.Likelihood(g, d, psd, w.modes, w.ns, w.t0, max_batch=64)
    yield w, psd, d, L
    L.close()
    torch.cuda.synchronize()


def test_sparse_stage_matches_oracle(small, oracle):
    w, psd, d, L = small
    print("case: sparse stage, small grid, 8 walkers", flush=True)
    B = L.waveform_gen(w.walkers)
    L.response(B)
    for i in range(B):
        g = L.get_sparse(i)
        o = oracle.sparse(w.walkers[i], w.grid, w.modes, w.ns, w.t0)
        assert np.array_equal(g["band"], o["band"]), (i, g["band"], o["band"])
        assert np.allclose(g["fband"], o["fband"], rtol=1e-14, atol=0)
        assert np.allclose(g["f"], o["f"], rtol=1e-14, atol=0)
        for q in range(8):
            scale = np.abs(o["fn"][:, q]).max(axis=1, keepdims=True) + 1e-300
            err = np.abs(g["fn"][:, q] - o["fn"][:, q]) / scale
            assert err.max() < 1e-11, (i, q, err.max())
        # spline coefficients: compare each term's size over its interval
        hpow = np.diff(o["f"], axis=1)[:, None, :, None] ** np.arange(4)
        scale = np.abs(o["fn"]).max(axis=2)[:, :, None, None] + 1e-300
        err = np.abs(g["cf"] - o["cf"]) * hpow / scale
        assert err.max() < 1e-10, (i, err.max())


def _compare_sparse(g, o, tag):
    """Band edges exactly; knots to 1e-14; amplitude and phase to 1e-11 of
    their own largest value over the mode; the six response functions (Re
    and Im of T^A, T^E, T^T) to 1e-11 of the mode's response scale, the
    largest of the six.  At low frequency T^T = (X + Y + Z) / sqrt(3) is a
    near-cancellation of terms of that scale (Sec. II, the A/E/T
    combinations), so its rounding is measured against them: relative to its
    own small values it can differ from the oracle by 1e-7 with both sides
    correct to rounding."""
    assert np.array_equal(g["band"], o["band"]), (tag, g["band"], o["band"])
    assert np.allclose(g["fband"], o["fband"], rtol=1e-14, atol=0), tag
    assert np.allclose(g["f"], o["f"], rtol=1e-14, atol=0), tag
    resp = np.abs(o["fn"][:, 2:8]).max(axis=(1, 2))[:, None] + 1e-300
    for q in range(8):
        scale = np.abs(o["fn"][:, q]).max(axis=1, keepdims=True) + 1e-300 if q < 2 else resp
        err = np.abs(g["fn"][:, q] - o["fn"][:, q]) / scale
        assert err.max() < 1e-11, (tag, q, err.max())


def test_band_edges_over_wide_mass_and_time_ranges(oracle):
    """The wavefront root searches (f_peak, each mode's f_start) against the
    oracle's halving, band edges bit for bit, over 96 walkers from 1e4 to
    3e8 solar masses and coalescence times from before the observation to
    after it, so that every outcome of the f_start search occurs: a mode
    already in band at the grid's first frequency, a start inside the band,
    and no band.  The batch takes the staged kernels; every fourth walker
    also goes through the fused one-walker kernel."""
    from paper_2005_01827_amd import mbh
    w = inputs.small_config(1, seed=7)
    g = w.grid
    T = 2.0 ** 20
    rng = np.random.default_rng(2024)
    n = 96
    th = np.empty((n, 11))
    th[:, 0] = np.exp(rng.uniform(math.log(1e4), math.log(3e8), n))
    th[:, 1] = rng.uniform(0.1, 1.0, n)
    th[:, 2:4] = rng.uniform(-0.9, 0.9, (n, 2))
    th[:, 4] = rng.uniform(1.0, 50.0, n)
    th[:, 5] = rng.uniform(0.0, 2 * math.pi, n)
    th[:, 6] = rng.uniform(0.05, math.pi - 0.05, n)
    th[:, 7] = rng.uniform(0.0, 2 * math.pi, n)
    th[:, 8] = rng.uniform(-1.5, 1.5, n)
    th[:, 9] = rng.uniform(0.0, math.pi, n)
    th[:, 10] = rng.uniform(-0.1 * T, 0.1 * T, n)
    th[::8, 10] = -0.95 * T                        # merged before the observation starts
    print(f"case: band edges, {n} walkers, M_T 1e4..3e8, small grid", flush=True)
    psd = inputs.psd_aet(g.freqs)
    d = inputs.noise(g, psd, 5)
    flo = g.k0 * g.df
    counts = dict(at_flo=0, inside=0, none=0)
    L = mbh.Likelihood(g, d, psd, w.modes, w.ns, w.t0, max_batch=n)
    L1 = mbh.Likelihood(g, d, psd, w.modes, w.ns, w.t0, max_batch=1)
    try:
        B = L.waveform_gen(th)
        L.response(B)
        for i in range(n):
            o = oracle.sparse(th[i], g, w.modes, w.ns, w.t0)
            _compare_sparse(L.get_sparse(i), o, i)
            for m in range(len(w.modes)):
                if not o["band"][m, 0]:
                    counts["none"] += 1
                elif o["fband"][m, 0] == flo:
                    counts["at_flo"] += 1
                else:
                    counts["inside"] += 1
            if i % 4 == 0:
                L1.loglike(th[i:i + 1])
                _compare_sparse(L1.get_sparse(0), o, ("fused", i))
    finally:
        L.close()
        L1.close()
    print(f"[band edges] mode outcomes {counts}", flush=True)
    assert min(counts.values()) >= 20, counts


def test_dense_stage_on_oracle_sparse_functions(small, oracle):
    """Dense interpolation + inner products fed the oracle's own knots and
    knot values: isolates the dense kernel and the device spline setup."""
    import torch
    w, psd, d, L = small
    print("case: dense stage on oracle sparse arrays, 8 walkers", flush=True)
    sps = [oracle.sparse(th, w.grid, w.modes, w.ns, w.t0) for th in w.walkers]
    B = L.set_sparse(np.stack([s["band"] for s in sps]), np.stack([s["fband"] for s in sps]),
                     np.stack([s["f"] for s in sps]), np.stack([s["fn"] for s in sps]))
    out = L.interp_and_inner(B)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = oracle.loglike(w.walkers, w.grid, d, psd, w.modes, w.ns, w.t0)
    _report("dense-on-oracle-sparse", got[:, 0], ref[:, 0])
    assert np.all(_lnl_close(got[:, 0], ref[:, 0]))
    hh = ref[:, 4:7].sum(1, keepdims=True)
    assert np.allclose(got[:, 1:], ref[:, 1:], rtol=0, atol=1e-10 * 10 * (hh + 1))


def test_loglike_small_grid_all_stages(small, oracle):
    import torch
    w, psd, d, L = small
    print("case: three stages, small grid, 8 walkers", flush=True)
    out = L.stages(w.walkers)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = oracle.loglike(w.walkers, w.grid, d, psd, w.modes, w.ns, w.t0)
    _report("stages-small", got[:, 0], ref[:, 0])
    assert np.all(_lnl_close(got[:, 0], ref[:, 0]))
    hh = ref[:, 4:7].sum(1, keepdims=True)
    assert np.allclose(got[:, 1:], ref[:, 1:], rtol=0, atol=1e-9 * (hh + 1))
    # the graph-launched entry point gives the same bits
    lnl = L.loglike(w.walkers)
    torch.cuda.synchronize()
    assert np.array_equal(lnl.cpu().numpy(), got[:, 0])


def test_determinism_and_batch_composition(small):
    import torch
    w, psd, d, L = small
    print("case: determinism / batch composition", flush=True)
    a = L.loglike(w.walkers).cpu().numpy()
    b = L.loglike(w.walkers).cpu().numpy()
    assert np.array_equal(a, b)
    perm = np.random.default_rng(1).permutation(len(w.walkers))
    big = np.concatenate([w.walkers[perm], w.walkers[:3]])
    c = L.loglike(big).cpu().numpy()
    assert np.array_equal(c[:len(perm)], a[perm])
    assert np.array_equal(c[len(perm):], a[:3])
    one = L.loglike(w.walkers[5:6]).cpu().numpy()
    assert np.array_equal(one, a[5:6])
    torch.cuda.synchronize()


def test_graph_follows_the_callers_buffers(small):
    """The captured graph reads the caller's parameter buffer and writes the
    caller's ln L buffer directly: launches back to back on one stream with
    alternating buffers (no synchronisation between them) give each buffer
    its own walkers' values, bitwise those of separate synchronised calls."""
    import torch
    w, psd, d, L = small
    print("case: graph launches on alternating caller buffers", flush=True)
    B = 6
    sets = [w.walkers[:B], w.walkers[2:2 + B], w.walkers[::-1][:B].copy()]
    ref = [L.loglike(x).cpu().numpy() for x in sets]
    p = [torch.as_tensor(x, dtype=torch.float64, device="cuda") for x in sets]
    o = [torch.full((B,), float("nan"), dtype=torch.float64, device="cuda") for _ in sets]
    for rep in range(3):
        for i in (0, 1, 2, 1, 0):
            L.loglike(p[i], out=o[i])
    torch.cuda.synchronize()
    for i in range(3):
        assert np.array_equal(o[i].cpu().numpy(), ref[i])
    # the same buffer with new contents is read afresh
    p[0].copy_(p[1])
    L.loglike(p[0], out=o[0])
    assert np.array_equal(o[0].cpu().numpy(), ref[1])


def test_schedules_give_identical_bits(small):
    """Every launch shape of the dense kernel (blocks per CU, one workgroup
    per walker) and the autotuner's choice give bitwise the same ln L."""
    import torch
    w, psd, d, L = small
    print("case: dense schedules / autotune", flush=True)
    ref = L.loglike(w.walkers).cpu().numpy()
    assert L.get_schedule() == (8, False)
    for bpc, one in ((1, False), (3, False), (16, False), (8, True)):
        L.set_schedule(bpc, one)
        assert L.get_schedule() == (bpc, one)
        assert np.array_equal(L.loglike(w.walkers).cpu().numpy(), ref)
    best, ms = L.autotune(w.walkers, reps=3)
    assert best in (2, 3, 4, 6, 8, 9, 12, 16, 24, 32) and ms > 0
    assert L.get_schedule() == (best, False)
    assert np.array_equal(L.loglike(w.walkers).cpu().numpy(), ref)
    L.set_schedule(8, False)
    torch.cuda.synchronize()


@pytest.mark.parametrize("modes,ns", [(((2, 2),), 8), (((2, 2), (3, 3)), 1024), (((4, 3), (2, 1)), 64)])
def test_mode_subsets_and_knot_counts(oracle, modes, ns):
    """Mode subsets (including the (2,2) mode alone and two higher modes
    without it) and the smallest and largest knot counts."""
    import torch
    from paper_2005_01827_amd import mbh
    print(f"case: modes={modes} ns={ns}", flush=True)
    w = inputs.small_config(6, seed=11)
    g = w.grid
    psd = inputs.psd_aet(g.freqs)
    d = oracle.template(w.injection, g, modes, ns, w.t0) + inputs.noise(g, psd, 78)
    L = mbh.Likelihood(g, d, psd, modes, ns, w.t0, max_batch=8)
    try:
        got = L.loglike(w.walkers).cpu().numpy()
        torch.cuda.synchronize()
        ref = oracle.loglike(w.walkers, g, d, psd, modes, ns, w.t0)
        _report(f"modes={len(modes)} ns={ns}", got, ref[:, 0])
        assert np.all(_lnl_close(got, ref[:, 0]))
    finally:
        L.close()


@pytest.mark.parametrize("ns", [8, 300, 560, 769, 1024])
def test_single_walker_fused_sparse_matches_batch(oracle, ns):
    """Small batches take the fused sparse kernel (the whole sparse stage in
    one launch; one walker also the dense kernel without an item list); the
    staged entry points take one kernel per step.  Knot counts chosen so the
    spline solves 8, 4, 2 and 1 functions per pass and leaves 1 to 64
    interleaved systems to the Thomas sweeps: each walker alone and the
    three together give bitwise the staged ln L, which matches the oracle."""
    import torch
    from paper_2005_01827_amd import mbh
    print(f"case: one walker against a batch, ns={ns}", flush=True)
    w = inputs.small_config(3, seed=13)
    g = w.grid
    psd = inputs.psd_aet(g.freqs)
    d = oracle.template(w.injection, g, w.modes, ns, w.t0) + inputs.noise(g, psd, 79)
    L = mbh.Likelihood(g, d, psd, w.modes, ns, w.t0, max_batch=4)
    try:
        batch = L.stages(w.walkers).cpu().numpy()[:, 0]
        fused = L.loglike(w.walkers).cpu().numpy()
        assert np.array_equal(fused, batch), (ns, fused, batch)
        for i in range(len(w.walkers)):
            one = L.loglike(w.walkers[i:i + 1]).cpu().numpy()
            assert np.array_equal(one, batch[i:i + 1]), (ns, i, one, batch[i])
        torch.cuda.synchronize()
        ref = oracle.loglike(w.walkers, g, d, psd, w.modes, ns, w.t0)
        _report(f"fused vs batch ns={ns}", batch, ref[:, 0])
        assert np.all(_lnl_close(batch, ref[:, 0]))
    finally:
        L.close()


def test_fused_threshold_bitwise(oracle):
    """Batches of up to 32 walkers take the fused sparse kernel, larger ones
    the chain of five kernels: the same walkers give the same bits either
    way (32 fused against 33 and 40 through the chain), and one of them
    matches the oracle."""
    import torch
    from paper_2005_01827_amd import mbh
    print("case: fused sparse threshold, 32 / 33 / 40 walkers", flush=True)
    w = inputs.small_config(40, seed=17)
    g = w.grid
    psd = inputs.psd_aet(g.freqs)
    d = oracle.template(w.injection, g, w.modes, w.ns, w.t0) + inputs.noise(g, psd, 81)
    L = mbh.Likelihood(g, d, psd, w.modes, w.ns, w.t0, max_batch=40)
    try:
        a = L.loglike(w.walkers[:32]).cpu().numpy()
        b = L.loglike(w.walkers[:33]).cpu().numpy()
        c = L.loglike(w.walkers).cpu().numpy()
        torch.cuda.synchronize()
    finally:
        L.close()
    assert np.array_equal(a, b[:32]) and np.array_equal(b, c[:33]), (a - b[:32], b - c[:33])
    ref = oracle.loglike(w.walkers[:2], g, d, psd, w.modes, w.ns, w.t0)
    assert np.all(_lnl_close(a[:2], ref[:, 0]))


def test_noiseless_injection_from_gpu_template_is_zero(small):
    import torch
    from paper_2005_01827_amd import mbh
    w, psd, d, L = small
    print("case: GPU template as data, lnL at injection", flush=True)
    h = L.template(w.injection).cpu().numpy()
    L2 = mbh.Likelihood(w.grid, h, psd, w.modes, w.ns, w.t0, max_batch=4)
    try:
        out = L2.stages(np.stack([w.injection, w.walkers[0]])).cpu().numpy()
        torch.cuda.synchronize()
        assert out[0, 0] == 0.0
        assert out[1, 0] < 0.0
    finally:
        L2.close()


def test_template_matches_oracle(small, oracle):
    w, psd, d, L = small
    print("case: dense template vs oracle", flush=True)
    h = L.template(w.walkers[2]).cpu().numpy()
    o = oracle.template(w.walkers[2], w.grid, w.modes, w.ns, w.t0)
    scale = np.abs(o).max()
    assert np.max(np.abs(h - o)) < 1e-9 * scale


def test_invalid_and_empty_walkers(small, oracle):
    import torch
    w, psd, d, L = small
    print("case: invalid / empty walkers", flush=True)
    th = np.repeat(w.injection[None], 5, axis=0)
    th[1, 1] = 1.5                      # q > 1
    th[2, 3] = 0.995                    # |a2| > 0.99
    th[3, 0] = float("nan")
    th[4, 0] = 1e9                      # ringdown below the band: no active mode
    out = L.stages(th).cpu().numpy()
    torch.cuda.synchronize()
    ref = oracle.loglike(th, w.grid, d, psd, w.modes, w.ns, w.t0)
    assert np.all(np.isneginf(out[1:4, 0]))
    assert np.all(_lnl_close(out[[0, 4], 0], ref[[0, 4], 0]))
    assert np.all(out[4, 1:] == 0.0)


def test_invalid_and_empty_walkers_alone(small, oracle):
    """The same edge cases one walker at a time (the single-walker item list):
    each matches its own row of a batched call, bit for bit."""
    import torch
    w, psd, d, L = small
    print("case: invalid / empty walkers, one per call", flush=True)
    th = np.repeat(w.injection[None], 5, axis=0)
    th[1, 1] = 1.5
    th[2, 3] = 0.995
    th[3, 0] = float("nan")
    th[4, 0] = 1e9
    batch = L.stages(th).cpu().numpy()
    lnl_batch = L.loglike(th).cpu().numpy()
    for i in range(len(th)):
        one = L.stages(th[i:i + 1]).cpu().numpy()
        assert np.array_equal(one[0], batch[i]) or (np.isneginf(one[0, 0]) and np.isneginf(batch[i, 0])), i
        lnl = L.loglike(th[i:i + 1]).cpu().numpy()
        assert np.array_equal(lnl, lnl_batch[i:i + 1]), i
    torch.cuda.synchronize()


def test_stage_order_is_enforced(oracle):
    """The staged calls refuse to run on a workspace that does not hold the
    preceding stage for the same B: a fresh context, a mismatched B, and a
    waveform stage without its response."""
    import torch
    from paper_2005_01827_amd import mbh
    print("case: stage order", flush=True)
    w = inputs.small_config(4, seed=7)
    g = w.grid
    psd = inputs.psd_aet(g.freqs)
    L = mbh.Likelihood(g, np.zeros((3, g.n), complex), psd, w.modes, w.ns, w.t0, max_batch=8)
    try:
        out7 = torch.empty((8, 7), dtype=torch.float64, device="cuda")
        ptr = ctypes.c_void_p(out7.data_ptr())
        assert L.lib.mbh_interp_and_inner(L.ctx, 4, ptr, None) == mbh.MBH_EINVAL
        assert L.lib.mbh_response(L.ctx, 4, None) == mbh.MBH_EINVAL
        assert L.lib.mbh_interp_and_inner(L.ctx, 0, ptr, None) == mbh.MBH_OK
        B = L.waveform_gen(w.walkers)
        assert L.lib.mbh_interp_and_inner(L.ctx, B, ptr, None) == mbh.MBH_EINVAL
        assert L.lib.mbh_response(L.ctx, B + 1, None) == mbh.MBH_EINVAL
        assert "mbh_waveform_gen" in L.lib.mbh_last_error(L.ctx).decode()
        L.response(B)
        assert L.lib.mbh_interp_and_inner(L.ctx, B - 1, ptr, None) == mbh.MBH_EINVAL
        a = L.interp_and_inner(B).cpu().numpy()
        # a full evaluation leaves its sparse stage for the inner products
        L.loglike(w.walkers[:2])
        b = L.interp_and_inner(2).cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(a[:2], b)
    finally:
        L.close()


def test_status_codes(small):
    from paper_2005_01827_amd import mbh
    w, psd, d, L = small
    with pytest.raises(mbh.MbhError) as e:
        L.loglike(np.repeat(w.injection[None], 65, axis=0))
    assert e.value.status == mbh.MBH_EBATCH
    assert L.lib.mbh_loglike_batch(L.ctx, None, 1, None, None) == mbh.MBH_EINVAL
    assert L.lib.mbh_loglike_batch(L.ctx, None, 0, None, None) == mbh.MBH_OK


def pick_walkers(L, B, n_even):
    """Walkers to check against the oracle: n_even evenly spaced, plus the
    shortest and the longest union band and the walker with the densest knots
    (the most knot crossings per dense step: active modes x intervals over
    its band length), from the device's own band table."""
    span = np.zeros(B)
    dens = np.zeros(B)
    for i in range(B):
        b = L.get_sparse(i)["band"]
        act = b[:, 0] == 1
        if act.any():
            span[i] = b[act, 2].max() - b[act, 1].min() + 1
            dens[i] = act.sum() * (L.n_sparse - 1) / span[i]
    has = np.flatnonzero(span > 0)
    extra = [] if has.size == 0 else [has[np.argmin(span[has])], has[np.argmax(span[has])],
                                      has[np.argmax(dens[has])]]
    idx = np.unique(np.concatenate([np.linspace(0, B - 1, n_even).astype(int), np.asarray(extra, dtype=int)]))
    return idx, span, dens


def _full_case(oracle, w, n_check, noise_seed, max_batch):
    import torch
    from paper_2005_01827_amd import mbh
    g = w.grid
    psd = inputs.psd_aet(g.freqs)
    h = oracle.template(w.injection, g, w.modes, w.ns, w.t0)
    d = h + inputs.noise(g, psd, noise_seed)
    L = mbh.Likelihood(g, d, psd, w.modes, w.ns, w.t0, max_batch=max_batch)
    try:
        got = L.loglike(w.walkers).cpu().numpy()
        torch.cuda.synchronize()
        idx, span, dens = pick_walkers(L, len(w.walkers), n_check)
        print(f"[{w.name}] checked {len(idx)} walkers; band spans {span[idx].min():.0f}..{span[idx].max():.0f} bins, "
              f"knot density up to {dens[idx].max():.3g} per bin", flush=True)
        ref = oracle.loglike(w.walkers[idx], g, d, psd, w.modes, w.ns, w.t0, nthreads=min(16, os.cpu_count()))
        _report(w.name, got[idx], ref[:, 0])
        assert np.all(_lnl_close(got[idx], ref[:, 0]))
        assert np.all(np.isfinite(got))
    finally:
        L.close()


def test_tobs22_full_grid(oracle):
    print("case: T_obs=2^22 grid, injection + 64 perturbations", flush=True)
    w = inputs.short_grid(65)
    w.walkers[0] = w.injection
    _full_case(oracle, w, 65, 101, 128)


@pytest.mark.slow
def test_tobs25_1024_walkers_sampled(oracle):
    print("case: T_obs=2^25 grid, 1024 walkers, 12 checked", flush=True)
    _full_case(oracle, inputs.year_grid(1024), 12, 2002, 1024)


@pytest.mark.slow
def test_uneven_batch_sampled(oracle):
    print("case: T_obs=2^25 grid, 2048 uneven walkers, 16 checked", flush=True)
    _full_case(oracle, inputs.uneven_batch(2048), 16, 2002, 2048)


def test_largest_batch_small_grid(oracle):
    """The largest batch a context accepts, 65536 walkers (about 35 GB of
    device workspace): every ln L finite and sampled walkers, first and last
    included, against the oracle."""
    import torch
    from paper_2005_01827_amd import mbh
    print("case: small grid, max_batch = 65536 walkers, 8 checked", flush=True)
    w = inputs.small_config(8, seed=7)
    g = w.grid
    psd = inputs.psd_aet(g.freqs)
    d = oracle.template(w.injection, g, w.modes, w.ns, w.t0) + inputs.noise(g, psd, 79)
    walkers = inputs.ball(w.injection, 1 << 16, 1e-3, 31)
    L = mbh.Likelihood(g, d, psd, w.modes, w.ns, w.t0, max_batch=1 << 16)
    try:
        got = L.loglike(walkers).cpu().numpy()
        torch.cuda.synchronize()
        idx = np.linspace(0, len(walkers) - 1, 8).astype(int)
        ref = oracle.loglike(walkers[idx], g, d, psd, w.modes, w.ns, w.t0)
        _report("max-batch-65536", got[idx], ref[:, 0])
        assert np.all(_lnl_close(got[idx], ref[:, 0]))
        assert np.all(np.isfinite(got))
    finally:
        L.close()


@pytest.mark.slow
def test_largest_knot_count_full_grid(oracle):
    """1024 knots per mode for all six modes on the T_obs = 2^25 s grid: the
    spline solve takes its four-functions-at-a-time path, and the dense stage
    sees the shortest intervals at full size."""
    import dataclasses
    print("case: T_obs=2^25 grid, ns = 1024, 6 modes, 16 walkers, 3 checked", flush=True)
    w = dataclasses.replace(inputs.year_grid(16), ns=1024)
    _full_case(oracle, w, 3, 2003, 16)
