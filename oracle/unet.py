"""FP64 CPU reference of the warm-start 3D U-Net (plain PyTorch CPU ops in float64).

Not in the paper: a learned initialiser for the Sec. 4.3 solver.  This module is
test infrastructure like the rest of ``oracle/``; it fixes the network's exact
definition so the GPU kernels can be checked layer by layer and gradient by
gradient.

Network (levels L = 4, widths w0..w3, 3x3x3 convolutions with zero padding 1):
  enc_l : x -> relu(conv(x)) -> relu(conv(.))          l = 0..3 (level 3 is the bottom)
  between levels: 2x2x2 average pooling
  dec_l : cat(skip_l, up2(coarse)) -> relu(conv) -> relu(conv)   l = 2..0
  head  : 1x1x1 convolution w0 -> 1 (no activation)
``up2`` repeats each voxel 2x2x2 (nearest).  Convolutions are cross-correlations
out[n] = b + sum_tap W[tap] in[n + d(tap)] (torch.nn.functional.conv3d).

Storage model (``bf16=True``): the network is specified with BF16 weights,
activations and activation gradients and FP32 (here: exact) sums.  The model rounds,
to the nearest BF16 with ties to even (of the value's FP32 rounding):
  values    -- the network input, every weight (biases stay unrounded), every
               post-ReLU convolution output and every pooled tensor;
  gradients -- of the head output, of every convolution input, of each encoder
               output that feeds both the skip and the pool (once, after the two
               contributions are summed) and of every tensor before upsampling
               (after the 8 children are summed).
Weight and bias gradients are not rounded.  With ``bf16=False`` everything is FP64.

Flat parameter layout shared with the device (``param_layout``): for each layer
in the order enc0a, enc0b, enc1a, enc1b, ..., dec0b, head: W as [Cout][tap][Cin]
with tap = (dx+1)*9 + (dy+1)*3 + (dz+1) (a single tap for the head), then the
bias [Cout].
"""
import numpy as np
import torch
import torch.nn.functional as F


def layer_specs(widths, in_ch=1):
    """(name, Cin, Cout, ksize) of every layer in parameter order."""
    w = list(widths)
    L = len(w)
    specs = []
    cin = in_ch
    for l in range(L):
        specs.append(("enc%da" % l, cin, w[l], 3))
        specs.append(("enc%db" % l, w[l], w[l], 3))
        cin = w[l]
    for l in range(L - 2, -1, -1):
        specs.append(("dec%da" % l, w[l] + w[l + 1], w[l], 3))
        specs.append(("dec%db" % l, w[l], w[l], 3))
    specs.append(("head", w[0], 1, 1))
    return specs


def param_layout(widths, in_ch=1):
    """[(name, cin, cout, k, w_offset, b_offset)], total count."""
    off = 0
    out = []
    for name, cin, cout, k in layer_specs(widths, in_ch):
        nw = cout * k ** 3 * cin
        out.append((name, cin, cout, k, off, off + nw))
        off += nw + cout
    return out, off


def unpack(flat, widths, in_ch=1):
    """Flat parameters -> {name: (weight [Cout, Cin, k, k, k], bias [Cout])} (torch f64)."""
    flat = torch.as_tensor(np.asarray(flat, dtype=np.float64))
    layout, total = param_layout(widths, in_ch)
    assert flat.numel() == total
    params = {}
    for name, cin, cout, k, wo, bo in layout:
        Wt = flat[wo:wo + cout * k ** 3 * cin].reshape(cout, k, k, k, cin).permute(0, 4, 1, 2, 3)
        params[name] = (Wt.contiguous(), flat[bo:bo + cout])
    return params


def pack_grads(grads, widths, in_ch=1):
    """{name: (dW [Cout,Cin,k,k,k], db)} -> flat array in the device layout."""
    layout, total = param_layout(widths, in_ch)
    out = np.zeros(total)
    for name, cin, cout, k, wo, bo in layout:
        dW, db = grads[name]
        out[wo:wo + cout * k ** 3 * cin] = dW.permute(0, 2, 3, 4, 1).reshape(-1).numpy()
        out[bo:bo + cout] = db.numpy()
    return out


def round_bf16(t):
    """Nearest BF16 (ties to even) of the FP32 rounding of t, held in float64."""
    return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def _store(t):
    """BF16 value with the gradient passed through unchanged."""
    return t + (round_bf16(t) - t).detach()


class _RoundGrad(torch.autograd.Function):
    """Identity whose backward rounds the incoming gradient to BF16."""

    @staticmethod
    def forward(ctx, t):
        return t.view_as(t)

    @staticmethod
    def backward(ctx, g):
        return round_bf16(g)


def forward(params, x, widths, bf16=False):
    """x: [X, Y, Z] or [Cin, X, Y, Z] -> output [X, Y, Z], float64 (with the BF16
    storage model of the module docstring if bf16)."""
    L = len(widths)
    val = _store if bf16 else (lambda t: t)
    grad = _RoundGrad.apply if bf16 else (lambda t: t)
    h = torch.as_tensor(x, dtype=torch.float64)
    if h.dim() == 3:
        h = h[None, None]
    elif h.dim() == 4:
        h = h[None]
    h = val(h)

    def conv(name, t, relu=True):
        W, b = params[name]
        k = W.shape[-1]
        y = F.conv3d(grad(t), val(W), b, padding=k // 2)
        return val(torch.relu(y)) if relu else y

    skips = []
    for l in range(L):
        if l:
            h = val(F.avg_pool3d(h, 2))
        h = conv("enc%db" % l, conv("enc%da" % l, h))
        if l < L - 1:
            h = grad(h)          # skip and pool gradients summed, then rounded
        skips.append(h)
    for l in range(L - 2, -1, -1):
        up = grad(h).repeat_interleave(2, 2).repeat_interleave(2, 3).repeat_interleave(2, 4)
        h = torch.cat([skips[l], up], dim=1)
        h = conv("dec%db" % l, conv("dec%da" % l, h))
    return grad(conv("head", h, relu=False))[0, 0]


def loss_and_grads(flat, x, target, widths, bf16=False):
    """MSE loss mean((net(x) - t)^2) and its gradient in the flat layout
    (x: [X, Y, Z] or [Cin, X, Y, Z]; t: [X, Y, Z]); bf16: the storage model of the
    module docstring."""
    in_ch = 1 if np.ndim(x) == 3 else np.shape(x)[0]
    params = unpack(flat, widths, in_ch)
    leaves = {}
    for k, (W, b) in params.items():
        W = W.clone().requires_grad_(True)
        b = b.clone().requires_grad_(True)
        leaves[k] = (W, b)
    y = forward(leaves, x, widths, bf16)
    t = torch.as_tensor(target, dtype=torch.float64)
    loss = torch.mean((y - t) ** 2)
    loss.backward()
    grads = {k: (W.grad, b.grad) for k, (W, b) in leaves.items()}
    return float(loss.detach()), pack_grads(grads, widths, in_ch), y.detach().numpy()


def conv3d_direct(x, W, b):
    """Direct-sum reference of one 3x3x3 zero-padded cross-correlation (pins conv3d).
    x [Cin, X, Y, Z], W [Cout, Cin, 3, 3, 3], b [Cout]."""
    cin, X, Y, Z = x.shape
    cout = W.shape[0]
    xp = np.zeros((cin, X + 2, Y + 2, Z + 2))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    out = np.zeros((cout, X, Y, Z))
    for co in range(cout):
        acc = np.full((X, Y, Z), b[co], dtype=np.float64)
        for ci in range(cin):
            for i in range(3):
                for j in range(3):
                    for k in range(3):
                        acc += W[co, ci, i, j, k] * xp[ci, i:i + X, j:j + Y, k:k + Z]
        out[co] = acc
    return out
