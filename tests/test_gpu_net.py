"""GPU warm-start network: BF16 MFMA layers and gradients against the FP64
reference network, the GPU training-data generator against a CPU twin on the same
Philox4x32-10 stream, and the gain of a briefly trained network over a cold start
at equal tolerance."""
import numpy as np
import pytest

from oracle import philox as oph
from oracle import unet
from gpu_util import announce, rel_l2, torch_cuda

pytestmark = pytest.mark.gpu
WIDTHS = (4, 8, 8, 16)


def _setup(seed=0, shape=(16, 16, 16), widths=WIDTHS, in_ch=1):
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    net = mh3d.Net(widths, in_channels=in_ch, seed=seed)
    rng = np.random.default_rng(seed)
    flat = np.zeros(net.nparam)
    lay, total = unet.param_layout(widths, in_ch)
    assert total == net.nparam
    for name, cin, cout, k, wo, bo in lay:      # He-normal weights, small biases
        flat[wo:bo] = rng.standard_normal(bo - wo) * np.sqrt(2.0 / (cin * k ** 3))
        flat[bo:bo + cout] = rng.standard_normal(cout) * 0.05
    net.set_params(torch.tensor(flat, dtype=torch.float32))
    x = rng.standard_normal(shape if in_ch == 1 else (in_ch,) + tuple(shape))
    t = rng.standard_normal(shape)
    return torch, net, flat, x, t


def _scale(x):
    """s = max |sum over channels| of the FP32 input."""
    x32 = x.astype(np.float32).astype(np.float64)
    return float(np.max(np.abs(x32 if x32.ndim == 3 else x32.sum(axis=0))))


def test_net_forward_matches_fp64_reference():
    """Against the reference network's BF16 storage model (the network's specified
    precision: BF16 weights and activations, FP32 sums) closely, and against its FP64
    form within the BF16 error."""
    torch, net, flat, x, t = _setup(1)
    announce("net forward")
    y = net.forward(torch.tensor(x, dtype=torch.float32)).cpu().numpy()
    s = _scale(x)
    params = unet.unpack(flat.astype(np.float32).astype(np.float64), WIDTHS)
    want = unet.forward(params, x / s, WIDTHS).numpy()
    model = unet.forward(params, x / s, WIDTHS, bf16=True).detach().numpy()
    print("forward rel err %.3e (FP64), %.3e (BF16 storage model)" % (rel_l2(y, want), rel_l2(y, model)), flush=True)
    assert rel_l2(y, model) <= 1e-4
    assert rel_l2(y, want) <= 3e-2


@pytest.mark.parametrize("widths,in_ch", [((8, 16), 1), ((16, 32), 3)])
def test_net_forward_reads_the_decoder_concatenation_in_place(widths, in_ch):
    """Inference runs the decoder's first convolution on [skip, upsampled coarse] read in
    place (strides 12, 24 and 48 with 4, 8 and 16 skip channels; the 4-level test net
    covers 12): the same values as the concatenated tensor, so the output meets the
    reference network's BF16 storage model as closely as with the concatenation."""
    torch, net, flat, x, t = _setup(4, shape=(16, 16, 16), widths=widths, in_ch=in_ch)
    announce("net forward, concatenation in place %s" % (widths,))
    y = net.forward(torch.tensor(x, dtype=torch.float32)).cpu().numpy()
    s = _scale(x)
    params = unet.unpack(flat.astype(np.float32).astype(np.float64), widths, in_ch)
    model = unet.forward(params, x / s, widths, bf16=True).detach().numpy()
    want = unet.forward(params, x / s, widths).numpy()
    assert rel_l2(y, model) <= 1e-4
    assert rel_l2(y, want) <= 3e-2


# The BF16 storage model rounds exactly where the device stores BF16, so the device
# and the model differ only by the order of the FP32 sums, which now and then moves a
# BF16 rounding by one ulp.  On the 2-level nets that leaves them equal to about 1e-7
# (bar 1e-4 per layer).  Through the 15 layers of the 4-level net such flips feed later
# rounding decisions, and the device and the model become two equally valid BF16
# realisations: each sits at the BF16 storage error from the FP64 network (the model
# measures it: 0.8 to 3.7 per cent per layer for this seed, the first layers' weight
# gradients being sums over all voxels with cancellation), so the bar there is 3e-2
# against the model and twice the measured storage error (+1e-2) against FP64.  A
# structural mistake (a wrong tap, channel or transpose) gives errors near 1.
@pytest.mark.parametrize("widths,shape,in_ch,model_tol", [((4, 8), (16, 16, 16), 1, 1e-4),
                                                          ((4, 8), (16, 8, 16), 5, 1e-4),
                                                          ((20, 8), (16, 16, 16), 1, 1e-4),   # channel strides 20, 28
                                                          ((24, 8), (8, 8, 8), 2, 1e-4),      # deep K on small grids
                                                          ((4, 8, 8, 16), (32, 32, 32), 3, 3e-2)])
def test_net_gradients_match_fp64_reference(widths, shape, in_ch, model_tol):
    torch, net, flat, x, t = _setup(2, shape=shape, widths=widths, in_ch=in_ch)
    announce("net gradients %s C=%d" % (widths, in_ch))
    loss = net.loss_grad(torch.tensor(x, dtype=torch.float32), torch.tensor(t, dtype=torch.float32))
    g = net.grads().cpu().numpy()
    s = _scale(x)
    f32 = flat.astype(np.float32).astype(np.float64)
    want_loss, want_g, _ = unet.loss_and_grads(f32, x / s, t / s, widths)
    model_loss, model_g, _ = unet.loss_and_grads(f32, x / s, t / s, widths, bf16=True)
    lay, _ = unet.param_layout(widths, in_ch)

    def per_layer(ref):
        return {name: (rel_l2(g[wo:bo], ref[wo:bo]), rel_l2(g[bo:bo + cout], ref[bo:bo + cout]))
                for name, cin, cout, k, wo, bo in lay}

    e_model, e_64 = per_layer(model_g), per_layer(want_g)
    e_storage = {name: (rel_l2(model_g[wo:bo], want_g[wo:bo]), rel_l2(model_g[bo:bo + cout], want_g[bo:bo + cout]))
                 for name, cin, cout, k, wo, bo in lay}
    fmt = lambda d: {k: "%.4f/%.4f" % v for k, v in d.items()}
    print("loss %.6e vs %.6e (FP64), %.6e (model); total grad rel err %.3e (FP64), %.3e (model)"
          % (loss, want_loss, model_loss, rel_l2(g, want_g), rel_l2(g, model_g)), flush=True)
    print("per layer (W/b) vs model: %s" % fmt(e_model), flush=True)
    print("per layer (W/b) vs FP64: %s" % fmt(e_64), flush=True)
    print("per layer (W/b) model vs FP64 (BF16 storage error): %s" % fmt(e_storage), flush=True)
    assert loss == pytest.approx(model_loss, rel=2e-3)
    assert loss == pytest.approx(want_loss, rel=2e-2)
    assert rel_l2(g, model_g) <= 1e-2
    assert rel_l2(g, want_g) <= 5e-2
    cos = float(np.dot(g, want_g) / (np.linalg.norm(g) * np.linalg.norm(want_g)))
    assert cos >= 0.998
    for name in e_model:
        assert e_model[name][0] <= model_tol and e_model[name][1] <= model_tol, name
        assert e_64[name][0] <= 2 * e_storage[name][0] + 1e-2, name
        assert e_64[name][1] <= 2 * e_storage[name][1] + 1e-2, name


def test_net_crop_uses_whole_volume_scale():
    torch, net, flat, x, t = _setup(3, shape=(32, 16, 16), in_ch=2)
    announce("net crop")
    crop = [8, 0, 0, 16, 16, 16]
    loss = net.loss_grad(torch.tensor(x, dtype=torch.float32), torch.tensor(t, dtype=torch.float32), crop)
    s = _scale(x)
    xc, tc = x[:, 8:24] / s, t[8:24] / s
    want_loss, want_g, _ = unet.loss_and_grads(flat.astype(np.float32).astype(np.float64), xc, tc, WIDTHS)
    assert loss == pytest.approx(want_loss, rel=3e-2)
    assert rel_l2(net.grads().cpu().numpy(), want_g) <= 5e-2


def _twin_phantom(shape, vox, seed, nsph, ntube):
    """CPU twin of the device phantom generator (same Philox stream and geometry)."""
    ext = [(n - 1) * vox for n in shape]
    key = (seed & 0xffffffff, seed >> 32)

    def u(obj, q):
        w = oph.philox4x32(np.array([q >> 2, obj, 0, 0], dtype=np.uint64), key)
        return (float(w[q & 3]) + 0.5) / 4294967296.0

    ax = [np.arange(n) * vox for n in shape]
    X, Y, Z = np.meshgrid(*ax, indexing="ij")
    out = np.zeros(shape)
    for i in range(nsph + ntube):
        if i < nsph:
            r = 2.0 + 3.0 * u(i, 0)
            c = [r + (ext[a] - 2 * r) * u(i, 1 + a) for a in range(3)]
            conc = 10.0 ** (-2.0 + 2.0 * u(i, 4))
            out += conc * (((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) <= r * r)
        else:
            r = 1.0 + 1.5 * u(i, 0)
            pts = np.array([3.0 + (ext[q % 3] - 6.0) * u(i, 1 + q) for q in range(9)]).reshape(3, 3)
            conc = 10.0 ** (-2.0 + 2.0 * u(i, 10))
            t = np.arange(257)[:, None] / 256.0
            curve = (1 - t) ** 2 * pts[0] + 2 * (1 - t) * t * pts[1] + t ** 2 * pts[2]
            P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], -1)
            best = np.full(len(P), np.inf)
            for s in range(len(curve)):
                best = np.minimum(best, np.sum((P - curve[s]) ** 2, axis=1))
            out += conc * (best <= r * r).reshape(shape)
    return out


def test_gpu_phantom_matches_cpu_twin_and_noise_hits_snr():
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    announce("phantom twin")
    shape = (24, 16, 12)
    p = mh3d.Plan(shape, (2, 3, 4), 1.2, (2, 2, 2), 10.0, 1e-3)
    got = p.phantom(12345, 5, 2).cpu().numpy()
    want = _twin_phantom(shape, 1.0, 12345, 5, 2)
    mism = np.abs(got - want) > 1e-5 * max(1.0, np.max(np.abs(want)))
    assert mism.mean() <= 1e-3 and np.max(np.abs(got - want)) <= 1.0 + 1e-6
    assert got.max() > 0
    # noise: empirical SNR per harmonic
    rho = p.phantom(7, 8, 1)
    clean = p.forward(rho).cpu().numpy().astype(np.float64)
    d = p.noisy_data(rho, 7, 30.0, 3.0).cpu().numpy().astype(np.float64)
    for i, k in enumerate((2, 3, 4)):
        noise = d[i] - clean[i]
        snr = 10 * np.log10(np.mean(clean[i] ** 2) / np.mean(noise ** 2))
        assert snr == pytest.approx(30.0 - 3.0 * (k - 2), abs=0.5)


def test_trained_network_saves_iterations():
    """A network trained for a few hundred GPU-generated samples starts the solver
    closer to the solution: fewer updates to the same stopping tolerance, and an end
    point no farther from the minimiser than the cold start's."""
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d, warmstart
    announce("warm-start gain")
    shape, harm = (32, 32, 32), (2, 3, 4, 5)
    p = mh3d.Plan(shape, harm, 1.2, (2, 2, 2), 20.0, 1e-3)
    net = mh3d.Net((8, 16, 16, 32), in_channels=len(harm), seed=11)
    hist = warmstart.train(p, net, 300, seed0=5_000_000, crop=shape, lr=2e-3, n_spheres=6, n_tubes=1,
                           log_every=50)
    assert hist[-1][1] < hist[0][1]
    res = warmstart.compare(p, net, [6_000_000 + j for j in range(4)], tol=1e-4, n_spheres=6, n_tubes=1)
    cold = np.mean([r["cold_iters"] for r in res])
    warm = np.mean([r["warm_iters"] for r in res])
    errs = []
    for r in res:
        ref, info = p.solve(r["d"], max_iter=20000, tol=1e-7, tau=0.0)
        assert info["rel_step"] <= 1e-7
        ref = ref.cpu().numpy()
        errs.append((rel_l2(r["cold"].cpu().numpy(), ref), rel_l2(r["warm"].cpu().numpy(), ref),
                     rel_l2(r["init"].cpu().numpy(), ref)))
    print("updates cold %.1f warm %.1f; distance to the minimiser (cold, warm, init): %s"
          % (cold, warm, ["%.3e/%.3e/%.3e" % e for e in errs]), flush=True)
    assert warm < cold
    for ec, ew, ei in errs:
        assert ei < 1.0          # the initialiser is closer than rho = 0
        assert ew <= 2.0 * ec + 1e-3
    # both end points reach about the same objective level (FP64 oracle evaluation).  The
    # stop at r_k <= 1e-4 bounds the step, not the objective gap, so the two end points are
    # different points on a slow descent: the bar is 5 % on the mean over the samples and
    # 10 % on each (the network itself, trained in BF16 for 300 steps, differs from build
    # to build with the order of its FP32 sums)
    from oracle import model as om
    from oracle import solver as osv
    op = osv.Operator(om.psf_bank(shape, list(harm), 1.2), om.sensitivity(shape, 20.0), (2, 2, 2), 1e-3)
    ratios = []
    for r in res:
        d = r["d"].cpu().numpy().astype(np.float64)
        fc = op.objective(r["cold"].cpu().numpy().astype(np.float64), d)
        fw = op.objective(r["warm"].cpu().numpy().astype(np.float64), d)
        print("objective cold %.6e warm %.6e" % (fc, fw), flush=True)
        ratios.append(fw / fc)
    assert np.mean(ratios) <= 1.05
    assert max(ratios) <= 1.10
