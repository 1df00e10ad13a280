"""Pins of the FP64 flow oracle against mathematics it does not compute itself:
finite differences, quadrature, the triangular-Jacobian identity, the
identity map and the closed-form first Adam step."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import flow_oracle as F
from paper_2005_01827_amd import inputs


def _flow(dim, L, H, scale, seed):
    perm = inputs.flow_perms(dim, L, seed)
    p = inputs.flow_params(F.num_params(dim, L, H), scale, seed + 1).astype(np.float64)
    return perm, p


def test_num_params_formula():
    # 11-D, 8 layers, H = 128: nc alternates 6/5, nt 5/6.
    H = 128
    per = lambda nc, nt: nc * H + H + H * H + H + H * 2 * nt + 2 * nt
    assert F.num_params(11, 8, H) == 4 * per(6, 5) + 4 * per(5, 6)


def test_identity_flow_is_standard_normal():
    dim, L, H = 5, 4, 16
    perm, p = _flow(dim, L, H, 0.3, 1)
    for l in F.unflatten(p, dim, L, H):        # views into p: zero W3 and b3
        l["W3"][...] = 0
        l["b3"][...] = 0
    u = np.random.default_rng(2).standard_normal((64, dim))
    z, logq = F.forward(p, u, perm, H)
    assert np.array_equal(z, u)
    ref = stats.multivariate_normal(np.zeros(dim), np.eye(dim)).logpdf(u)
    assert np.allclose(logq, ref, rtol=0, atol=1e-12)


def test_inverse_undoes_forward_and_agrees_on_logq():
    dim, L, H = 11, 6, 32
    perm, p = _flow(dim, L, H, 0.4, 3)
    u = np.random.default_rng(4).standard_normal((200, dim)) * 1.5
    z, lq_f = F.forward(p, u, perm, H)
    assert np.abs(z - u).max() > 0.1                # the map is not trivial
    u2, lq_i = F.inverse(p, z, perm, H)
    assert np.allclose(u2, u, rtol=0, atol=1e-11)
    assert np.allclose(lq_i, lq_f, rtol=0, atol=1e-11)


def test_logdet_equals_finite_difference_jacobian():
    """log q(u) + |z|^2/2 + (dim/2) ln 2pi must equal ln|det dz/du|."""
    dim, L, H = 11, 4, 16
    perm, p = _flow(dim, L, H, 0.5, 5)
    u0 = np.random.default_rng(6).standard_normal((5, dim))
    z0, lq = F.forward(p, u0, perm, H)
    h = 1e-5
    for r in range(len(u0)):
        J = np.empty((dim, dim))
        for j in range(dim):
            up = u0[r].copy(); up[j] += h
            um = u0[r].copy(); um[j] -= h
            J[:, j] = (F.forward(p, up[None], perm, H)[0][0] - F.forward(p, um[None], perm, H)[0][0]) / (2 * h)
        sign, ld = np.linalg.slogdet(J)
        assert sign > 0
        ld_oracle = lq[r] + 0.5 * z0[r] @ z0[r] + 0.5 * dim * math.log(2 * math.pi)
        assert abs(ld - ld_oracle) < 1e-7


def test_density_integrates_to_one_in_two_dimensions():
    dim, L, H = 2, 4, 16
    perm, p = _flow(dim, L, H, 0.6, 7)
    g = np.linspace(-30, 30, 3001)                 # the tails reach |u| ~ 20
    X, Y = np.meshgrid(g, g, indexing="ij")
    u = np.stack([X.ravel(), Y.ravel()], axis=1)
    _, logq = F.forward(p, u, perm, H)
    dx = g[1] - g[0]
    assert abs(np.exp(logq).sum() * dx * dx - 1.0) < 1e-6


def test_gradient_matches_central_differences():
    dim, L, H = 4, 3, 8
    perm, p = _flow(dim, L, H, 0.5, 9)
    u = np.random.default_rng(10).standard_normal((32, dim))
    loss, g = F.loss_grad(p, u, perm, H)
    _, lq = F.forward(p, u, perm, H)
    assert abs(loss + lq.mean()) < 1e-13
    h = 1e-6
    idx = np.random.default_rng(11).choice(len(p), 60, replace=False)
    # Include entries of the last linear maps, which start every gradient.
    off = F.num_params(dim, L, H) - 2 * (dim - F.layer_nc(dim, L - 1))
    idx = np.concatenate([idx, [off, off + 1, len(p) - 1]])
    for i in idx:
        pp = p.copy(); pp[i] += h
        pm = p.copy(); pm[i] -= h
        fd = (F.loss_grad(pp, u, perm, H)[0] - F.loss_grad(pm, u, perm, H)[0]) / (2 * h)
        assert abs(fd - g[i]) < 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_adam_first_step_closed_form():
    """After one step from zero moments, mhat = g and vhat = g^2, so every
    parameter moves by lr * g / (|g| + eps)."""
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    p0 = np.array([1.0, 2.0, 3.0, 4.0])
    p1, m, v = F.adam(p0, g, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(p1, p0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # A second identical gradient keeps mhat = g and vhat = g^2.
    p2, _, _ = F.adam(p1, g, m, v, 2, 0.01)
    assert np.allclose(p2 - p1, p1 - p0, rtol=1e-12, atol=1e-15)


def test_layer_split_follows_the_documented_layout():
    """Layer l keeps perm_l[:ceil(dim/2)] for even l and perm_l[:floor(dim/2)]
    for odd l unchanged; the other coordinates move."""
    dim, L, H = 7, 2, 8
    perm, p = _flow(dim, L, H, 0.5, 13)
    u = np.random.default_rng(14).standard_normal((16, dim))
    for keep_layer in range(L):
        q = p.copy()
        for l, d in enumerate(F.unflatten(q, dim, L, H)):
            if l != keep_layer:
                d["W3"][...] = 0
                d["b3"][...] = 0
        z, _ = F.forward(q, u, perm, H)
        nc = (dim + 1) // 2 if keep_layer % 2 == 0 else dim // 2
        kept, moved = perm[keep_layer][:nc], perm[keep_layer][nc:]
        assert np.array_equal(z[:, kept], u[:, kept])
        assert np.all(np.abs(z[:, moved] - u[:, moved]).max(axis=0) > 1e-3)
