"""Training and use of the warm-start network (driver only: every step runs in the
library's kernels -- phantoms, forward model, noise, back-projection, network
forward/backward and Adam)."""
import math
import time

import numpy as np

from . import mh3d


def sample_snr2(seed, lo=20.0, hi=40.0):
    """SNR of the 2nd harmonic for training sample `seed` (3 dB/harmonic decay after)."""
    return float(np.random.default_rng([seed, 3]).uniform(lo, hi))


def crop_origin(seed, shape, crop):
    rng = np.random.default_rng([seed, 4])
    return [int(rng.integers(0, n - c + 1)) for n, c in zip(shape, crop)]


def learning_rate(j, steps, lr, lr_final=None):
    """Step j of `steps`: lr, or a cosine decay from lr (j = 0) to lr_final (last step)."""
    if lr_final is None:
        return lr
    return lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * j / max(1, steps - 1)))


def train(plan, net, steps, seed0=5_000_000, crop=(64, 64, 64), lr=1e-3, n_spheres=80, n_tubes=6,
          snr=(20.0, 40.0), decay_db=3.0, log=None, log_every=100, target="phantom", crops_per_sample=1,
          solve_tol=1e-4, solve_max_iter=5000, lr_final=None, evaluate=None, eval_at=()):
    """Trains `net` on `steps` crops of phantom/portrait pairs generated on the GPU from
    the plan's forward model (sample j uses seed seed0 + j; each sample serves
    crops_per_sample consecutive steps).  target "phantom" regresses the phantom;
    "solution" regresses the plain solver's end point at solve_tol from rho = 0 (the
    point a warm-started solve converges to).  Returns the loss history (every
    log_every steps).  lr_final: cosine decay of the learning rate from lr to lr_final
    over the steps (constant lr if None).  evaluate(j): called before step j for every j
    in eval_at (and after the last step if steps is in eval_at), e.g. a validation loss."""
    hist = []
    eval_at = set(int(j) for j in eval_at)
    t0 = time.perf_counter()
    x = tgt = None
    for j in range(steps):
        if evaluate is not None and j in eval_at:
            evaluate(j)
        sample = j // crops_per_sample
        seed = seed0 + sample
        if j % crops_per_sample == 0:
            rho = plan.phantom(seed, n_spheres, n_tubes)
            d = plan.noisy_data(rho, seed, sample_snr2(seed, *snr), decay_db)
            x = plan.backproject(d)
            if target == "solution":
                tgt, _ = plan.solve(d, max_iter=solve_max_iter, tol=solve_tol, tau=0.0)
            else:
                tgt = rho
        want = (j % log_every == 0) or (j == steps - 1)
        o = crop_origin(seed * 131 + j % crops_per_sample, plan.shape, crop)
        loss = net.loss_grad(x, tgt, list(o) + list(crop), want_loss=want)
        net.adam_step(learning_rate(j, steps, lr, lr_final))
        if want:
            hist.append((j, loss))
            if log:
                log("train step %d/%d loss %.4e (%.1f s)" % (j, steps, loss, time.perf_counter() - t0))
    if evaluate is not None and steps in eval_at:
        evaluate(steps)
    return hist


def validation_loss(plan, net, samples):
    """Mean over held-out (back-projection, phantom) pairs of the training loss on the
    whole volume, mean((net(x/s) - rho/s)^2) with s = max |A^T d| (network forward only;
    the mean runs in torch on the device)."""
    torch = plan.torch
    tot = 0.0
    for x, rho in samples:
        y = net.forward(x)
        s = float(x.sum(dim=0).abs().max())
        tot += float(torch.mean((y - rho / s) ** 2))
    return tot / max(1, len(samples))


def compare(plan, net, seeds, tol=1e-4, max_iter=5000, n_spheres=80, n_tubes=6, snr=(20.0, 40.0), decay_db=3.0):
    """Cold vs warm-started solves on held-out samples; both refined to the same
    r_k <= tol.  Returns per-sample dicts."""
    torch = plan.torch
    out = []
    for seed in seeds:
        rho = plan.phantom(seed, n_spheres, n_tubes)
        d = plan.noisy_data(rho, seed, sample_snr2(seed, *snr), decay_db)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cold, ic = plan.solve(d, max_iter=max_iter, tol=tol, tau=0.0)
        torch.cuda.synchronize()
        t_cold = time.perf_counter() - t0
        t0 = time.perf_counter()
        init = net.warm_start(plan, d)
        warm, iw = plan.solve(d, rho0=init, max_iter=max_iter, tol=tol, tau=0.0)
        torch.cuda.synchronize()
        t_warm = time.perf_counter() - t0
        out.append({"seed": seed, "cold_iters": ic["iters"], "warm_iters": iw["iters"], "cold_s": t_cold,
                    "warm_s": t_warm, "cold": cold, "warm": warm, "init": init, "truth": rho, "d": d})
    return out
