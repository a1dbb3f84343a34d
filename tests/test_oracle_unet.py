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
