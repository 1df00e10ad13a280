"""GPU parity of the learned-proposal flow kernels against the FP64 oracle.

The kernels run in FP32.  Tolerances: a dot product of length K in FP32
errs by about sqrt(K) * 2^-24 * sum|w_i h_i| in typical cases; with K <= 128,
|h| <= 1 and weights U(-0.15, 0.15) that is ~1e-6 per MLP output, amplified
through 8 layers by the exp(s) scales (|s| < 1) to well under 1e-4 on z.
The tests allow 2e-4 absolute + 2e-5 relative on coordinates and 1e-3 on
log q, which the measured errors stay an order of magnitude below.
"""
import math

import numpy as np
import pytest

from oracle import flow_oracle as F
from paper_2005_01827_amd import inputs

pytestmark = pytest.mark.gpu

DIM, L, H = 11, 8, 128


@pytest.fixture(scope="module")
def mbh():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_01827_amd import mbh as M
    return M


def _setup(mbh, scale=0.15, seed=21, max_batch=32768, dim=DIM, nl=L, hid=H):
    perm = inputs.flow_perms(dim, nl, seed)
    fl = mbh.Flow(dim, nl, hid, max_batch, perm=perm, seed=seed)
    assert fl.n_params == F.num_params(dim, nl, hid)
    p = inputs.flow_params(fl.n_params, scale, seed + 1)
    fl.set_params(p)
    return fl, perm, p


def _rows(n, dim, seed, scale=1.3):
    return (np.random.default_rng(seed).standard_normal((n, dim)) * scale).astype(np.float32)


def test_layout_and_params_roundtrip(mbh):
    fl, perm, p = _setup(mbh)
    perm2, nc = fl.layout()
    assert np.array_equal(perm2, perm)
    assert list(nc) == [F.layer_nc(DIM, l) for l in range(L)]
    assert np.array_equal(fl.get_params(), p)
    fl.close()


def test_default_init_is_identity(mbh):
    fl = mbh.Flow(DIM, L, H, 1024, seed=5)
    u = _rows(100, DIM, 1)
    z, lq = fl.forward(u)
    assert np.array_equal(z.cpu().numpy(), u)
    ref = -0.5 * (u.astype(np.float64) ** 2).sum(1) - 0.5 * DIM * math.log(2 * math.pi)
    assert np.allclose(lq.cpu().numpy(), ref, rtol=0, atol=2e-5)
    fl.close()


@pytest.mark.parametrize("n", [1, 17, 1000])
def test_forward_matches_oracle(mbh, n):
    fl, perm, p = _setup(mbh)
    u = _rows(n, DIM, 100 + n)
    z, lq = fl.forward(u)
    z_ref, lq_ref = F.forward(p.astype(np.float64), u.astype(np.float64), perm, H)
    z, lq = z.cpu().numpy().astype(np.float64), lq.cpu().numpy().astype(np.float64)
    ez = np.abs(z - z_ref) / (2e-4 + 2e-5 * np.abs(z_ref))
    print(f"n={n}: max |dz| {np.abs(z - z_ref).max():.2e}, max |dlogq| {np.abs(lq - lq_ref).max():.2e}")
    assert np.abs(z_ref - u).max() > 0.05
    assert ez.max() < 1.0
    assert np.abs(lq - lq_ref).max() < 1e-3
    fl.close()


def test_inverse_matches_oracle_and_undoes_forward(mbh):
    fl, perm, p = _setup(mbh)
    z = _rows(999, DIM, 7, scale=1.0)
    u, lq = fl.inverse(z)
    u_ref, lq_ref = F.inverse(p.astype(np.float64), z.astype(np.float64), perm, H)
    u_np, lq = u.cpu().numpy().astype(np.float64), lq.cpu().numpy().astype(np.float64)
    print(f"inverse: max |du| {np.abs(u_np - u_ref).max():.2e}, max |dlogq| {np.abs(lq - lq_ref).max():.2e}")
    assert (np.abs(u_np - u_ref) / (2e-4 + 2e-5 * np.abs(u_ref))).max() < 1.0
    assert np.abs(lq - lq_ref).max() < 1e-3
    z2, lq2 = fl.forward(u)
    assert np.abs(z2.cpu().numpy() - z).max() < 2e-4
    assert np.abs(lq2.cpu().numpy() - lq).max() < 1e-3
    fl.close()


@pytest.mark.parametrize("dim,nl,hid", [(7, 3, 40), (32, 2, 16), (5, 1, 256)])
def test_other_shapes_match_oracle(mbh, dim, nl, hid):
    """Layer widths that are not a multiple of the kernels' 16-weight load
    batches (40), the smallest (16) and largest (256) widths, the widest
    input (32: 16 kept coordinates, 32 outputs per layer) and one layer:
    forward, inverse and the gradient against the FP64 oracle."""
    fl, perm, p = _setup(mbh, dim=dim, nl=nl, hid=hid, max_batch=4096)
    p64 = p.astype(np.float64)
    u = _rows(333, dim, 41 + dim)
    z, lq = fl.forward(u)
    z_ref, lq_ref = F.forward(p64, u.astype(np.float64), perm, hid)
    z, lq = z.cpu().numpy().astype(np.float64), lq.cpu().numpy().astype(np.float64)
    print(f"dim {dim} L {nl} H {hid}: max |dz| {np.abs(z - z_ref).max():.2e}, "
          f"max |dlogq| {np.abs(lq - lq_ref).max():.2e}")
    assert np.abs(z_ref - u).max() > 0.05
    assert (np.abs(z - z_ref) / (2e-4 + 2e-5 * np.abs(z_ref))).max() < 1.0
    assert np.abs(lq - lq_ref).max() < 1e-3
    zz = _rows(77, dim, 43 + dim, scale=1.0)
    uu, lqi = fl.inverse(zz)
    u_ref, lqi_ref = F.inverse(p64, zz.astype(np.float64), perm, hid)
    assert (np.abs(uu.cpu().numpy() - u_ref) / (2e-4 + 2e-5 * np.abs(u_ref))).max() < 1.0
    assert np.abs(lqi.cpu().numpy() - lqi_ref).max() < 1e-3
    loss, g = fl.loss_grad(u)
    loss_ref, g_ref = F.loss_grad(p64, u.astype(np.float64), perm, hid)
    assert abs(loss - loss_ref) < 1e-4 * max(1.0, abs(loss_ref))
    assert np.abs(g.astype(np.float64) - g_ref).max() < 2e-4 * np.abs(g_ref).max()
    fl.close()


@pytest.mark.parametrize("n", [777, 20000])
def test_loss_and_gradient_match_oracle(mbh, n):
    """777 rows: 3 full 256-row chunks and a ragged one; 20000 rows: 64
    chunks of 313 rows, the last one ragged."""
    fl, perm, p = _setup(mbh)
    u = _rows(n, DIM, 300 + n)
    loss, g = fl.loss_grad(u)
    loss_ref, g_ref = F.loss_grad(p.astype(np.float64), u.astype(np.float64), perm, H)
    gmax = np.abs(g_ref).max()
    err = np.abs(g.astype(np.float64) - g_ref)
    cos = g @ g_ref / (np.linalg.norm(g) * np.linalg.norm(g_ref))
    print(f"n={n}: loss {loss:.9f} ref {loss_ref:.9f}; max grad err {err.max():.2e} of max |g| {gmax:.2e}; "
          f"cos {cos:.9f}")
    assert abs(loss - loss_ref) < 1e-4 * max(1.0, abs(loss_ref))
    assert err.max() < 2e-4 * gmax
    assert cos > 1 - 1e-7
    # Deterministic: a second call is bitwise identical.
    loss2, g2 = fl.loss_grad(u)
    assert loss2 == loss and np.array_equal(g2, g)
    fl.close()


def test_adam_steps_follow_the_update_rule(mbh):
    fl, perm, p0 = _setup(mbh)
    u = _rows(512, DIM, 9)
    lr = 1e-3
    _, g1 = fl.loss_grad(u)
    fl.adam(lr)
    p1 = fl.get_params()
    _, g2 = fl.loss_grad(u)
    fl.adam(lr)
    p2 = fl.get_params()
    g1, g2 = g1.astype(np.float64), g2.astype(np.float64)
    step1 = lr * g1 / (np.abs(g1) + 1e-8)
    assert np.abs((p0 - p1) - step1).max() < 1e-6 * lr + 2e-7 * np.abs(p0).max()
    m = 0.1 * 0.9 * g1 + 0.1 * g2
    v = 0.001 * 0.999 * g1 * g1 + 0.001 * g2 * g2
    step2 = lr * (m / (1 - 0.81)) / (np.sqrt(v / (1 - 0.999 ** 2)) + 1e-8)
    assert np.abs((p1.astype(np.float64) - p2) - step2).max() < 1e-5 * lr + 2e-7 * np.abs(p1).max()
    fl.close()


def test_training_learns_a_curved_density(mbh):
    """Maximum likelihood on banana-shaped samples: the trained flow must beat
    the best Gaussian (whose loss is the Gaussian entropy) clearly."""
    x = inputs.banana(20000, DIM, 11)
    mu, sd = x.mean(0), x.std(0)
    u = ((x - mu) / sd).astype(np.float32)
    gauss = 0.5 * DIM * (1 + math.log(2 * math.pi)) + 0.5 * np.linalg.slogdet(np.corrcoef(u.T))[1]
    fl = mbh.Flow(DIM, L, H, 4096, seed=3)
    import torch
    ud = torch.as_tensor(u, device="cuda")
    rng = np.random.default_rng(4)
    for _ in range(400):
        idx = torch.as_tensor(rng.integers(0, len(u), 4096), device="cuda")
        loss, _ = fl.loss_grad(ud.index_select(0, idx), want_grad=False)
        fl.adam(2e-3)
    full = []
    for b in range(0, len(u), 4096):
        _, lq = fl.forward(u[b:b + 4096])
        full.append(lq.cpu().numpy())
    nll = -np.concatenate(full).astype(np.float64).mean()
    print(f"trained NLL {nll:.4f} vs best Gaussian {gauss:.4f}")
    assert nll < gauss - 0.3
    fl.close()


def test_rejects_bad_arguments(mbh):
    M = mbh
    with pytest.raises(M.MbhError):
        M.Flow(1, 8, 128, 16)
    with pytest.raises(M.MbhError):
        M.Flow(DIM, 8, 128, 16, perm=np.zeros((8, DIM), dtype=np.int32))   # not permutations
    fl = M.Flow(DIM, 2, 32, 16, seed=1)
    with pytest.raises(M.MbhError):
        fl.forward(np.zeros((17, DIM), np.float32))                      # beyond max_batch
    with pytest.raises(M.MbhError):
        fl.adam(1e-3)                                                    # no gradient yet
    fl.close()


def test_training_recovers_a_known_gaussian(mbh):
    """Trained on draws of a correlated Gaussian, the flow's own samples must
    reproduce its mean and covariance, and its NLL must approach the entropy."""
    import torch
    rng = np.random.default_rng(12)
    A = rng.standard_normal((DIM, DIM)) / math.sqrt(DIM)
    cov = A @ A.T + 0.3 * np.eye(DIM)
    mu = rng.standard_normal(DIM)
    x = rng.multivariate_normal(mu, cov, 40000)
    from paper_2005_01827_amd.sampler import FlowProposal
    prop = FlowProposal(DIM, max_batch=32768, seed=13, defensive=0.0)
    prop.fit(x, steps=400, lr=2e-3, batch=4096, seed=14, val_frac=0.0)
    xs, lq = prop.sample(20000, np.random.default_rng(15))
    entropy = 0.5 * DIM * (1 + math.log(2 * math.pi)) + 0.5 * np.linalg.slogdet(cov)[1]
    nll = -prop.logq(x[:20000]).mean()
    se = np.sqrt(np.diag(cov) / len(xs))
    print(f"NLL {nll:.4f} vs entropy {entropy:.4f}; max |mean err|/se "
          f"{(np.abs(xs.mean(0) - mu) / se).max():.2f}")
    assert nll < entropy + 0.05
    assert np.all(np.abs(xs.mean(0) - mu) < 6 * se)
    assert np.abs(np.cov(xs.T) - cov).max() < 0.05 * np.abs(cov).max()
    # log q of a draw, re-evaluated from the stored float64 point (float32
    # standardization twice), agrees to float32 rounding
    assert np.allclose(lq, prop.logq(xs), rtol=0, atol=1e-4)
    prop.flow.close()
