"""Pins of the FP64 CNN oracle: convolution against torch's float64 CPU
conv2d (a library routine), the adjoints against torch autograd and central
finite differences on a tiny network."""
import numpy as np
import torch

import oracle


def test_conv_matches_torch_library():
    rng = np.random.default_rng(0)
    for C, H, W in ((8, 12, 16), (5, 7, 9)):
        x = rng.normal(size=(2, C, H, W)); w = rng.normal(size=(6, C, 3, 3)); b = rng.normal(size=6)
        ref = torch.nn.functional.conv2d(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b), stride=2,
                                         padding=1).numpy()
        np.testing.assert_allclose(oracle.conv2d(x, w, b), ref, rtol=1e-12, atol=1e-12)


def test_conv_adjoints_match_torch_autograd():
    rng = np.random.default_rng(1)
    x = torch.from_numpy(rng.normal(size=(2, 4, 9, 11))).requires_grad_()
    w = torch.from_numpy(rng.normal(size=(5, 4, 3, 3))).requires_grad_()
    b = torch.from_numpy(rng.normal(size=5)).requires_grad_()
    y = torch.nn.functional.conv2d(x, w, b, stride=2, padding=1)
    g = torch.from_numpy(rng.normal(size=tuple(y.shape)))
    (y * g).sum().backward()
    dx, dw, db = oracle.conv2d_bwd(x.detach().numpy(), w.detach().numpy(), g.numpy())
    np.testing.assert_allclose(dx, x.grad.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(dw, w.grad.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(db, b.grad.numpy(), rtol=1e-12, atol=1e-12)


def tiny_params(rng, cin=2, ch=3):
    p = {}
    c = cin
    for l in range(4):
        p[f"w{l}"] = rng.normal(0, 0.5, size=(ch, c, 3, 3)); p[f"b{l}"] = rng.normal(0, 0.1, size=ch)
        c = ch
    p["wfc"] = rng.normal(0, 0.5, size=(6, 3 * ch)); p["bfc"] = rng.normal(0, 0.1, size=6)
    return p


def test_network_gradient_finite_differences():
    """FD on a 2-channel toy network (FP64)."""
    rng = np.random.default_rng(2)
    p = tiny_params(rng)
    x = rng.normal(size=(2, 2, 16, 16))
    lab = rng.normal(size=(2, 6))
    scale = np.array([1, 1, 1, 2, 2, 2.0])

    def L(pp):
        out, _ = oracle.initnet_forward(x, pp)
        return oracle.initnet_loss(out, lab, scale)[0]

    out, cache = oracle.initnet_forward(x, p)
    _, dout = oracle.initnet_loss(out, lab, scale)
    grads = oracle.initnet_backward(p, cache, dout)
    checked = 0
    for name, arr in p.items():
        flat = arr.reshape(-1)
        for i in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            h = 1e-6
            old = flat[i]
            flat[i] = old + h; lp = L(p)
            flat[i] = old - h; lm = L(p)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = grads[name].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, i, fd, an)
            checked += 1
    assert checked > 40


def test_moment_pooling_closed_forms():
    """The head's pooled values: a map that is constant per channel has zero
    first moments (the pixel centres are symmetric about 0) and its value as
    the mean; a map equal to x^ has the mean of x^ squared as its x^-moment,
    (1 - 1/w^2) / 3 for the w centres (2 x + 1) / w - 1."""
    for h, w in ((8, 10), (3, 5)):
        basis = oracle.moment_basis(h, w)
        assert abs(basis[1].sum()) < 1e-12 and abs(basis[2].sum()) < 1e-12
        np.testing.assert_allclose((basis[1] ** 2).mean(), (1 - 1 / w ** 2) / 3, rtol=1e-12)
        np.testing.assert_allclose((basis[2] ** 2).mean(), (1 - 1 / h ** 2) / 3, rtol=1e-12)
    # through the network: zero convolution weights, bias only, so the last map
    # is the constant relu(b3) per channel; the head sees [relu(b3), 0, 0]
    rng = np.random.default_rng(4)
    p = tiny_params(rng, cin=2, ch=3)
    for l in range(4):
        p[f"w{l}"][:] = 0.0
    out, (acts, pool) = oracle.initnet_forward(rng.normal(size=(1, 2, 16, 16)), p)
    np.testing.assert_allclose(pool[0], np.concatenate([np.maximum(p["b3"], 0), np.zeros(6)]), atol=1e-15)
    np.testing.assert_allclose(out[0], p["wfc"][:, :3] @ np.maximum(p["b3"], 0) + p["bfc"], rtol=1e-12)
