"""The likelihood entry point that allocates nothing
(mbh_loglike_batch_noalloc), called through the C ABI, against the
graph-launched mbh_loglike_batch on the same context: the same kernels in the
same order, so ln L must agree bit for bit.  Two calls in a row, the second
with a smaller batch (the fixed per-GPU workspace keeps the first call's
contents), on the small grid and on the 2^25-s grid; a batch whose workspace
exceeds the fixed array is refused with MBH_EBATCH."""
import ctypes

import numpy as np
import pytest

from paper_2005_01827_amd import inputs

pytestmark = pytest.mark.gpu


def _noalloc(L, p_dev, out_dev):
    """Direct C-ABI call; returns the status."""
    import torch
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return L.lib.mbh_loglike_batch_noalloc(L.ctx, ctypes.c_void_p(p_dev.data_ptr()), p_dev.shape[0],
                                           ctypes.c_void_p(out_dev.data_ptr()), s)


def _two_calls(L, walkers, sizes, label):
    import torch
    from paper_2005_01827_amd import mbh
    for B in sizes:
        print(f"case: {label}, noalloc B={B}", flush=True)
        p = torch.as_tensor(walkers[:B], dtype=torch.float64, device="cuda").contiguous()
        out = torch.full((B,), float("nan"), dtype=torch.float64, device="cuda")
        st = _noalloc(L, p, out)
        assert st == mbh.MBH_OK, L.lib.mbh_last_error(L.ctx)
        got = out.cpu().numpy()
        ref = L.loglike(p).cpu().numpy()
        torch.cuda.synchronize()
        print(f"[{label} B={B}] noalloc {got[:3]} graph {ref[:3]}", flush=True)
        assert np.array_equal(got, ref, equal_nan=False), (got, ref)


def test_noalloc_matches_graph_small_grid(oracle):
    import torch
    from paper_2005_01827_amd import mbh
    w = inputs.small_config(16, seed=7)
    g = w.grid
    psd = inputs.psd_aet(g.freqs)
    d = oracle.template(w.injection, g, w.modes, w.ns, w.t0) + inputs.noise(g, psd, 77)
    walkers = w.walkers.copy()
    walkers[3, 1] = np.nan            # an invalid walker: -inf on both paths
    L = mbh.Likelihood(g, d, psd, w.modes, w.ns, w.t0, max_batch=16)
    try:
        _two_calls(L, walkers, (16, 5), "small grid")
        # a later call with a different batch again, and B = 0 (no-op)
        _two_calls(L, walkers[::-1].copy(), (9,), "small grid, reversed")
        p0 = torch.empty((0, 11), dtype=torch.float64, device="cuda")
        o0 = torch.empty(1, dtype=torch.float64, device="cuda")
        assert _noalloc(L, p0, o0) == mbh.MBH_OK
        # one walker against the oracle as well
        p = torch.as_tensor(w.walkers[:2], dtype=torch.float64, device="cuda").contiguous()
        out = torch.empty(2, dtype=torch.float64, device="cuda")
        assert _noalloc(L, p, out) == mbh.MBH_OK
        got = out.cpu().numpy()
        ref = oracle.loglike(w.walkers[:2], g, d, psd, w.modes, w.ns, w.t0)[:, 0]
        assert np.all(np.abs(got - ref) <= 1e-10 * np.maximum(np.abs(ref), 1.0)), (got, ref)
        # warm calls leave the device's free memory unchanged
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        for _ in range(3):
            assert _noalloc(L, p, out) == mbh.MBH_OK
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        assert free1 == free0, (free0, free1)
    finally:
        L.close()


def test_noalloc_matches_graph_tobs25_and_refuses_oversize(oracle):
    import torch
    from paper_2005_01827_amd import mbh
    w = inputs.year_grid(256)
    g = w.grid
    psd = inputs.psd_aet(g.freqs)
    d = oracle.template(w.injection, g, w.modes, w.ns, w.t0) + inputs.noise(g, psd, 2002)
    L = mbh.Likelihood(g, d, psd, w.modes, w.ns, w.t0, max_batch=256)
    try:
        _two_calls(L, w.walkers, (96, 40), "2^25-s grid")
        print("case: 2^25-s grid, noalloc B=256 (over the fixed workspace)", flush=True)
        p = torch.as_tensor(w.walkers, dtype=torch.float64, device="cuda").contiguous()
        out = torch.empty(256, dtype=torch.float64, device="cuda")
        st = _noalloc(L, p, out)
        msg = L.lib.mbh_last_error(L.ctx).decode()
        print(f"[2^25-s grid B=256] status {st}: {msg}", flush=True)
        assert st == mbh.MBH_EBATCH and "static workspace" in msg
        # the context still works after the refusal
        _two_calls(L, w.walkers[100:], (8,), "2^25-s grid after refusal")
    finally:
        L.close()
