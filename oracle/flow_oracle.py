"""FP64 CPU oracle of the affine-coupling flow used as the learned proposal.

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU baseline of
the benchmark use this module; the product path never imports it.

The flow is the density model behind the independence proposal that the
sampler mixes with the stretch move (Sec. III.A: affine-invariant ensemble
sampling with parallel tempering; the learned proposal is the extension the
method's throughput makes affordable).  It is a stack of affine coupling
layers (the real-valued non-volume-preserving construction: half of the
coordinates condition an elementwise affine map of the other half, so the
Jacobian is triangular and its log-determinant is the sum of the log-scales).

Definition computed here, written out plainly in float64:
  layer l: x_c = x[perm_l[:nc_l]], x_t = x[perm_l[nc_l:]]
           h1 = tanh(x_c W1 + b1); h2 = tanh(h1 W2 + b2); o = h2 W3 + b3
           s = tanh(o[:nt]); t = o[nt:]
           y[perm_l[nc_l:]] = x_t * exp(s) + t; y[perm_l[:nc_l]] = x_c
  z = f(u);  log q(u) = -|z|^2/2 - (dim/2) log(2 pi) + sum over layers of sum s
  loss = -(1/n) sum_i log q(u_i); its gradient comes from torch autograd.
nc_l = ceil(dim/2) for even l and floor(dim/2) for odd l.  Parameters are a
flat array, per layer W1[nc][H], b1[H], W2[H][H], b2[H], W3[H][2nt], b3[2nt]
(each weight input-major).

Pins (tests/test_oracle_flow.py): the gradient against central finite
differences, the log-determinant against the finite-difference Jacobian,
inverse(forward(u)) == u, normalization of q by quadrature in two
dimensions, and the identity flow reducing to the standard normal.
"""
import math

import numpy as np
import torch


def layer_nc(dim, layer):
    return (dim + 1) // 2 if layer % 2 == 0 else dim // 2


def layer_shapes(dim, n_layers, hidden):
    """[(nc, nt, [(name, shape), ...]), ...] in flat-array order."""
    out = []
    for l in range(n_layers):
        nc = layer_nc(dim, l)
        nt = dim - nc
        out.append((nc, nt, [("W1", (nc, hidden)), ("b1", (hidden,)), ("W2", (hidden, hidden)),
                             ("b2", (hidden,)), ("W3", (hidden, 2 * nt)), ("b3", (2 * nt,))]))
    return out


def num_params(dim, n_layers, hidden):
    return sum(int(np.prod(s)) for _, _, names in layer_shapes(dim, n_layers, hidden) for _, s in names)


def unflatten(params, dim, n_layers, hidden):
    """Split a flat tensor into per-layer dicts of views (keeps autograd)."""
    layers, off = [], 0
    for nc, nt, names in layer_shapes(dim, n_layers, hidden):
        d = {"nc": nc, "nt": nt}
        for name, shape in names:
            size = int(np.prod(shape))
            d[name] = params[off:off + size].reshape(shape)
            off += size
        layers.append(d)
    assert off == len(params)
    return layers


def _mlp(p, xc):
    h1 = torch.tanh(xc @ p["W1"] + p["b1"])
    h2 = torch.tanh(h1 @ p["W2"] + p["b2"])
    o = h2 @ p["W3"] + p["b3"]
    nt = p["nt"]
    return torch.tanh(o[:, :nt]), o[:, nt:]


def _forward_t(params, u, perm, hidden):
    dim = u.shape[1]
    layers = unflatten(params, dim, len(perm), hidden)
    x = u
    logdet = torch.zeros(u.shape[0], dtype=u.dtype)
    for l, p in enumerate(layers):
        pc = list(perm[l][:p["nc"]])
        pt = list(perm[l][p["nc"]:])
        s, t = _mlp(p, x[:, pc])
        y = x.clone()
        y[:, pt] = x[:, pt] * torch.exp(s) + t
        x = y
        logdet = logdet + s.sum(dim=1)
    logq = -0.5 * (x * x).sum(dim=1) - 0.5 * dim * math.log(2 * math.pi) + logdet
    return x, logq


def _as64(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64))


def forward(params, u, perm, hidden):
    """z = f(u) and log q(u); numpy in, numpy float64 out."""
    with torch.no_grad():
        z, logq = _forward_t(_as64(params), _as64(u), np.asarray(perm), hidden)
    return z.numpy(), logq.numpy()


def inverse(params, z, perm, hidden):
    """u = f^{-1}(z) and log q(u), undoing the layers in reverse order."""
    z = _as64(z)
    dim = z.shape[1]
    perm = np.asarray(perm)
    layers = unflatten(_as64(params), dim, len(perm), hidden)
    y = z.clone()
    logdet = torch.zeros(z.shape[0], dtype=z.dtype)
    with torch.no_grad():
        for l in range(len(layers) - 1, -1, -1):
            p = layers[l]
            pc = list(perm[l][:p["nc"]])
            pt = list(perm[l][p["nc"]:])
            s, t = _mlp(p, y[:, pc])
            x = y.clone()
            x[:, pt] = (y[:, pt] - t) * torch.exp(-s)
            y = x
            logdet = logdet + s.sum(dim=1)
    logq = -0.5 * (z * z).sum(dim=1) - 0.5 * dim * math.log(2 * math.pi) + logdet
    return y.numpy(), logq.numpy()


def loss_grad(params, u, perm, hidden):
    """(-(1/n) sum log q(u_i), d loss / d params) in float64."""
    p = _as64(params).clone().requires_grad_(True)
    _, logq = _forward_t(p, _as64(u), np.asarray(perm), hidden)
    loss = -logq.mean()
    loss.backward()
    return float(loss.detach()), p.grad.numpy().copy()


def adam(params, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam update; returns (params, m, v) as new arrays.
    step is the 1-based count of this update."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mhat = m / (1 - b1 ** step)
    vhat = v / (1 - b2 ** step)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v
