"""Pins for the FP64 reference U-Net of the warm start (oracle/unet.py)."""
import numpy as np
import pytest
import torch

from oracle import unet

WIDTHS = (2, 4, 8, 16)


def _flat(seed, widths=WIDTHS):
    lay, tot = unet.param_layout(widths)
    rng = np.random.default_rng(seed)
    return rng.standard_normal(tot) * 0.3


def test_conv3d_matches_direct_sum():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 5, 4, 6))
    W = rng.standard_normal((2, 3, 3, 3, 3))
    b = rng.standard_normal(2)
    got = torch.nn.functional.conv3d(torch.tensor(x)[None], torch.tensor(W), torch.tensor(b), padding=1)[0].numpy()
    assert np.max(np.abs(got - unet.conv3d_direct(x, W, b))) < 1e-12


def test_layout_round_trip_and_count():
    lay, tot = unet.param_layout((8, 16, 32, 80))
    assert tot == 455073
    flat = _flat(1)
    params = unet.unpack(flat, WIDTHS)
    back = unet.pack_grads(params, WIDTHS)
    assert np.array_equal(back, flat)
    # W[co][tap][ci] with tap = (dx+1)*9 + (dy+1)*3 + (dz+1)
    name, cin, cout, k, wo, bo = lay[1]
    flat8 = _flat(2, (8, 16, 32, 80))
    W = unet.unpack(flat8, (8, 16, 32, 80))[name][0]
    co, ci, tap = 3, 5, 2 * 9 + 0 * 3 + 1
    assert W[co, ci, 2, 0, 1] == flat8[wo + (co * 27 + tap) * cin + ci]


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((8, 8, 8))
    t = rng.standard_normal((8, 8, 8))
    flat = _flat(4)
    loss, grad, _ = unet.loss_and_grads(flat, x, t, WIDTHS)
    idx = rng.choice(len(flat), 40, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(flat)
        e[i] = h
        lp, _, _ = unet.loss_and_grads(flat + e, x, t, WIDTHS)
        lm, _, _ = unet.loss_and_grads(flat - e, x, t, WIDTHS)
        fd = (lp - lm) / (2 * h)
        assert fd == pytest.approx(grad[i], rel=1e-6, abs=1e-9)


def test_shapes_and_skips():
    flat = _flat(5)
    y = unet.forward(unet.unpack(flat, WIDTHS), np.ones((16, 8, 8)), WIDTHS)
    assert tuple(y.shape) == (16, 8, 8)


def test_multichannel_input_gradient_matches_finite_differences():
    widths = (2, 4)
    lay, tot = unet.param_layout(widths, in_ch=3)
    assert lay[0][1] == 3 and tot == unet.param_layout(widths)[1] + 2 * 27 * 2
    rng = np.random.default_rng(6)
    x = rng.standard_normal((3, 8, 4, 8))
    t = rng.standard_normal((8, 4, 8))
    flat = rng.standard_normal(tot) * 0.3
    loss, grad, y = unet.loss_and_grads(flat, x, t, widths)
    assert y.shape == (8, 4, 8)
    # channel c of the input only meets the weights W[:, c] of the first layer
    idx = list(rng.choice(lay[0][5] - lay[0][4], 12, replace=False)) + list(rng.choice(tot, 12, replace=False))
    h = 1e-6
    for i in idx:
        e = np.zeros_like(flat)
        e[i] = h
        lp, _, _ = unet.loss_and_grads(flat + e, x, t, widths)
        lm, _, _ = unet.loss_and_grads(flat - e, x, t, widths)
        assert (lp - lm) / (2 * h) == pytest.approx(grad[i], rel=1e-6, abs=1e-9)


def _bf(a):
    """Nearest BF16 (ties to even) of the FP32 rounding of a, from the bit pattern."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def test_round_bf16_ties_to_even():
    v = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8 + 2.0 ** -20), 3.0, 2.0 ** -130])
    want = np.array([1.0, 1.0 + 2.0 ** -6, -(1.0 + 2.0 ** -7), 3.0, 2.0 ** -130])
    assert np.array_equal(unet.round_bf16(torch.tensor(v)).numpy(), want)
    assert np.array_equal(_bf(v), want)


def _conv(x, W, b):
    return unet.conv3d_direct(x, W, b)


def _conv_t(g, W):
    """Input gradient of a 3x3x3 zero-padded cross-correlation: dx[ci, n] = sum W[co, ci, t] g[co, n - d(t)]."""
    cout, cin = W.shape[:2]
    X, Y, Z = g.shape[1:]
    gp = np.zeros((cout, X + 2, Y + 2, Z + 2))
    gp[:, 1:-1, 1:-1, 1:-1] = g
    dx = np.zeros((cin, X, Y, Z))
    for co in range(cout):
        for ci in range(cin):
            for i in range(3):
                for j in range(3):
                    for k in range(3):
                        dx[ci] += W[co, ci, i, j, k] * gp[co, 2 - i:2 - i + X, 2 - j:2 - j + Y, 2 - k:2 - k + Z]
    return dx


def _conv_w(x, g):
    """Weight gradient: dW[co, ci, t] = sum_n g[co, n] x[ci, n + d(t)]."""
    cin, X, Y, Z = x.shape
    xp = np.zeros((cin, X + 2, Y + 2, Z + 2))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    dW = np.zeros((g.shape[0], cin, 3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                dW[:, :, i, j, k] = np.einsum("oxyz,cxyz->oc", g, xp[:, i:i + X, j:j + Y, k:k + Z])
    return dW


def _pool(a):
    c, X, Y, Z = a.shape
    return a.reshape(c, X // 2, 2, Y // 2, 2, Z // 2, 2).mean(axis=(2, 4, 6))


def _up(a):
    return a.repeat(2, 1).repeat(2, 2).repeat(2, 3)


def _sum8(a):
    c, X, Y, Z = a.shape
    return a.reshape(c, X // 2, 2, Y // 2, 2, Z // 2, 2).sum(axis=(2, 4, 6))


def test_bf16_storage_model_matches_step_by_step_two_level_net():
    """The BF16 storage model of the reference network against a hand-written forward
    and backward of a 2-level net (every rounding point written out; numpy only)."""
    widths = (2, 3)
    rng = np.random.default_rng(8)
    lay, tot = unet.param_layout(widths)
    flat = (rng.standard_normal(tot) * 0.4).astype(np.float32).astype(np.float64)
    x = rng.standard_normal((4, 4, 4))
    t = rng.standard_normal((4, 4, 4))
    loss, grad, y = unet.loss_and_grads(flat, x, t, widths, bf16=True)
    P = {k: (W.numpy(), b.numpy()) for k, (W, b) in unet.unpack(flat, widths).items()}
    Wq = {k: _bf(W) for k, (W, b) in P.items()}
    relu = lambda a: np.maximum(a, 0.0)
    # forward
    x0 = _bf(x)[None]
    ea0 = _bf(relu(_conv(x0, Wq["enc0a"], P["enc0a"][1])))
    es0 = _bf(relu(_conv(ea0, Wq["enc0b"], P["enc0b"][1])))
    p1 = _bf(_pool(es0))
    ea1 = _bf(relu(_conv(p1, Wq["enc1a"], P["enc1a"][1])))
    es1 = _bf(relu(_conv(ea1, Wq["enc1b"], P["enc1b"][1])))
    cat0 = np.concatenate([es0, _up(es1)])
    da0 = _bf(relu(_conv(cat0, Wq["dec0a"], P["dec0a"][1])))
    db0 = _bf(relu(_conv(da0, Wq["dec0b"], P["dec0b"][1])))
    yy = np.einsum("c,cxyz->xyz", Wq["head"][0, :, 0, 0, 0], db0) + P["head"][1][0]
    assert np.allclose(y, yy, rtol=0, atol=1e-12)
    assert loss == pytest.approx(np.mean((yy - t) ** 2), rel=1e-12)
    # backward
    g = {}
    gy = _bf(2.0 * (yy - t) / yy.size)
    g["head"] = (np.einsum("xyz,cxyz->c", gy, db0)[None, :, None, None, None], np.array([gy.sum()]))
    g_db0 = _bf(Wq["head"][0, :, 0, 0, 0][:, None, None, None] * gy[None])

    def layer(name, gout, act, inp):
        gp = gout * (act > 0)
        g[name] = (_conv_w(inp, gp), gp.sum(axis=(1, 2, 3)))
        return _bf(_conv_t(gp, Wq[name]))

    g_da0 = layer("dec0b", g_db0, db0, da0)
    g_cat = layer("dec0a", g_da0, da0, cat0)
    g_es1 = _bf(_sum8(g_cat[widths[0]:]))
    g_ea1 = layer("enc1b", g_es1, es1, ea1)
    g_p1 = layer("enc1a", g_ea1, ea1, p1)
    g_es0 = _bf(g_cat[:widths[0]] + _up(g_p1) / 8.0)
    g_ea0 = layer("enc0b", g_es0, es0, ea0)
    layer("enc0a", g_ea0, ea0, x0)
    want = unet.pack_grads({k: (torch.tensor(a), torch.tensor(b)) for k, (a, b) in g.items()}, widths)
    assert np.linalg.norm(grad - want) <= 1e-10 * np.linalg.norm(want)
    # and the model is a BF16-sized perturbation of the FP64 network, not another network
    _, g64, y64 = unet.loss_and_grads(flat, x, t, widths)
    assert 1e-5 < np.linalg.norm(y - y64) / np.linalg.norm(y64) < 3e-2
