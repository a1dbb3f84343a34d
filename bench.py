"""Benchmark of the MH3D hot path on one MI355X.

A step is one application of the forward operator A followed by its adjoint A^T
applied to A's output (Sec. 4.1 eq. dN; each accelerated-projected-gradient update of
Sec. 4.3 costs one of each) on the workload's resident inputs: d = A rho is written to
HBM and x = A^T d is computed in three launches: the forward plane pass, one class pass
doing the forward and adjoint spectral products of its alias classes (as the solver's
updates do), and one launch running the adjoint plane pass beside the small-grid pass
that writes d.  The rate of the two separate calls (six launches) is reported beside
it.  The JSON line reports A+A^T applications per second, the HBM roofline of the dominant kernel (measured with
HIP events around its launches), the FP64 CPU oracle timed on a bounded sample of
the same workload, and the time to reconstruct at r_k <= 1e-4 with the plain solver
(data and the zero start image resident in HBM; the first call includes the power
iteration for the step size, the second reuses it).

The batched leg solves the 64 uneven volumes of the batch workload (sizes 48^3 ..
128x128x96, 2..10 harmonics) to r_k <= 1e-4 each, once as 64 sequential plain
solves and once as one batched solve, and reports both wall times.

The warm-start leg trains the 3D U-Net on GPU-generated phantom/portrait pairs of
the warm-start workload (128^3, k = 2..12, SNR_2 ~ U(20, 40) dB, 64^3 crops), then
solves held-out samples to r_k <= 1e-4 from rho = 0 and from the network's output
(inference included in the warm wall time), and reports iterations, wall times and
the distance of both end points to the phantom.

The cpu_baseline leg (the only one that runs the FP64 oracle) times the oracle's
A+A^T and its reconstruction of oracle-made data, which the GPU solver repeats on the
same data: the relative L2 difference of the two reconstructions is reported there.

The vector leg times the same fused step for the vector model of eq. matrixModel on
the workload's grid (seeded synthetic component PSFs and sensitivities, C = 1 and 3).
The MH2D leg does the same, and a solve to r_k <= 1e-4, for the 2D projection geometry
of Sec. 5.2 (128 x 256 image, two scans of seven harmonics).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 1|2] [--no-cpu] [--no-solve]
                       [--no-batch] [--no-warm] [--no-vector] [--no-mh2d] [--warm-train-steps T]
                       [--warm-eval E]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def algorithmic_bytes(w, compact=True, ncomp=1):
    """Per-application algorithmic bytes of A (and of A^T, the same total):
    4N (rho) + 4CN (b) + beta_H C K N_c (spectra) + 4 K M (portraits); of one
    separate class pass: beta_H C K N_c + 8 C N_c (yz spectra in) + 8 K M_c
    (decimated spectra out); and of the fused class pass (forward and adjoint in one):
    beta_H C K N_c (spectra, read once) + 16 C N_c (yz spectra in and out) + 8 K M_c
    (decimated spectra out, or the data's in for the solver's residual).
    N_c = nx ny (nz/2+1), M_c = mx my (mz/2+1), C the components of the vector model
    (1 for the scalar model)."""
    nx, ny, nz = w.shape
    mx, my, mz = w.small_shape
    K = len(w.harmonics)
    N = nx * ny * nz
    M = mx * my * mz
    Nc = nx * ny * (nz // 2 + 1)
    Mc = mx * my * (mz // 2 + 1)
    bh = 4 if compact else 8
    C = ncomp
    op = 4 * N + 4 * C * N + bh * C * K * Nc + 4 * K * M
    spectral = bh * C * K * Nc + 8 * C * Nc + 8 * K * Mc
    fused = bh * C * K * Nc + 16 * C * Nc + 8 * K * Mc
    return op, spectral, fused


def class_roofline(pass_us, w, compact=True, ncomp=1):
    """The dominant class kernel of the A+A^T step: the fused class pass where the plan
    runs one, else the average of the forward and adjoint class passes.  Returns
    (kernel label, algorithmic bytes per launch, seconds per launch)."""
    _, spectral, fused = algorithmic_bytes(w, compact, ncomp)
    if "class_normal" in pass_us:
        return "class_normal (forward + adjoint spectral products and alias folds)", fused, \
            pass_us["class_normal"] * 1e-6
    return "class_fwd+class_adj (spectral multiply + alias fold)", spectral, \
        0.5 * (pass_us["class_fwd"] + pass_us["class_adj"]) * 1e-6


def cpu_baseline(w, rho, r, plan=None, budget_s=12.0):
    """The FP64 oracle (FFT tier, scipy.fft with all host cores) on the same workload:
    full A+A^T applications until the time budget is used (the rate), then -- when a
    plan is given -- the oracle's own reconstruction of oracle-made data (its power
    iteration and FISTA to the workload's r_k), which the GPU solver repeats on the
    same data with the oracle's tau: both update counts and their relative L2
    difference are reported."""
    import numpy as np
    from oracle import model as om
    from oracle import philox as oph
    from oracle import solver as osv
    from paper_2503_13802_amd import inputs
    t0 = time.perf_counter()
    h = om.psf_bank(w.shape, list(w.harmonics), w.a_per_mm, w.voxel_mm)
    b = om.sensitivity(w.shape, w.sigma_mm, w.voxel_mm)
    setup = time.perf_counter() - t0
    n = 0
    t0 = time.perf_counter()
    while True:
        om.forward_fft(h, b, rho, w.ds)
        om.adjoint_fft(h, b, r, w.ds)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 50:
            break
    out = {"value": n / el, "unit": "A+A^T applications/s", "cores": os.cpu_count(), "kind": "oracle",
           "sample": "%d full A+A^T applications of the FP64 FFT-tier oracle (scipy.fft, workers=%d) on the "
                     "same workload; PSF/sensitivity setup %.1f s excluded" % (n, os.cpu_count(), setup)}
    if plan is not None:
        import torch
        op = osv.Operator(h, b, w.ds, w.lam)
        t0 = time.perf_counter()
        d = inputs.add_noise(op.A(rho), w.snr_db, r)
        tau = osv.step_size(osv.power_iteration(op, oph.uniform01(0, 0, w.n_voxels).reshape(w.shape), 50))
        want, _, n_o = osv.fista(op, d, tau, max_iter=w.max_iter, tol=w.tol)
        solve_s = time.perf_counter() - t0
        got, info = plan.solve(torch.tensor(d, dtype=torch.float32, device="cuda"), max_iter=w.max_iter,
                               tol=w.tol, tau=tau)
        got = got.cpu().numpy().astype(np.float64)
        out["reconstruction"] = {
            "oracle_s": round(solve_s, 2), "oracle_iters": int(n_o), "gpu_iters": info["iters"], "tau": tau,
            "gpu_vs_oracle_rel_l2": float(np.linalg.norm(got - want) / np.linalg.norm(want)),
            "note": "oracle-made data (phantom + noise of the workload), oracle power iteration for tau, "
                    "both solvers stop at r_k <= %g" % w.tol}
    return out


def batched_leg(batch_inputs, tol, max_iter, tile_cache=None):
    """64 uneven volumes to r_k <= tol: sequential plain solves vs one batched solve."""
    import numpy as np
    import torch
    from paper_2503_13802_amd import inputs, mh3d
    bws, phantoms, _ = batch_inputs
    dev = torch.device("cuda:0")
    plans, ds = [], []
    for bw, ph in zip(bws, phantoms):
        p = mh3d.Plan(bw.shape, bw.harmonics, bw.a_per_mm, bw.ds, bw.sigma_mm, bw.lam, bw.voxel_mm)
        if tile_cache is not None:
            p.autotune(tile_cache)
        clean = p.forward(torch.tensor(ph, dtype=torch.float32, device=dev)).cpu().numpy().astype(np.float64)
        d = inputs.add_noise(clean, bw.snr_db, inputs.noise_draw(bw))
        plans.append(p)
        ds.append(torch.tensor(d, dtype=torch.float32, device=dev))
    torch.cuda.synchronize()
    log("batched leg: %d plans built" % len(plans))
    # untimed: the batch's graphs and every plan's step size (power iteration, cached
    # per plan), then a first plain solve (kernel code loading) on the first volume
    batch = mh3d.Batch(plans)
    t0 = time.perf_counter()
    batch.solve(ds, max_iter=16, tol=0.0, tau=0.0)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    plans[0].solve(ds[0], max_iter=20, tol=0.0, tau=0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq = [p.solve(d, max_iter=max_iter, tol=tol, tau=0.0) for p, d in zip(plans, ds)]
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    rhos, infos = batch.solve(ds, max_iter=max_iter, tol=tol, tau=0.0)
    torch.cuda.synchronize()
    bat_s = time.perf_counter() - t0
    same = all(torch.equal(r, s[0]) for r, s in zip(rhos, seq))
    iters_seq = [s[1]["iters"] for s in seq]
    iters_bat = [i["iters"] for i in infos]
    conv = sum(1 for i in infos if i["rel_step"] <= tol)
    vox = sum(int(np.prod(bw.shape)) for bw in bws)
    return {"volumes": len(plans), "voxels": vox, "sequential_s": round(seq_s, 4), "batched_s": round(bat_s, 4),
            "speedup": round(seq_s / bat_s, 3), "converged": conv, "iters_max": max(iters_bat),
            "iters_mean": round(float(np.mean(iters_bat)), 1), "identical_to_sequential": bool(same),
            "iters_match": iters_seq == iters_bat, "step_size_setup_s": round(setup_s, 4),
            "note": "step sizes (50 batched power iterations per volume) computed once, untimed, for both forms"}


def warm_leg(train_steps, n_eval, tol, max_iter, tile_cache=None):
    """Warm-start workload: GPU training, then cold vs warm solves on held-out seeds."""
    import numpy as np
    import torch
    from paper_2503_13802_amd import inputs, mh3d, warmstart
    w = inputs.workload(4)
    plan = mh3d.Plan(w.shape, w.harmonics, w.a_per_mm, w.ds, w.sigma_mm, w.lam, w.voxel_mm)
    if tile_cache is not None:
        plan.autotune(tile_cache)
    net = mh3d.Net((8, 16, 32, 80), in_channels=len(w.harmonics), seed=w.seed)
    log("warm leg: %s, network %d parameters, training %d steps" % (w.name, net.nparam, train_steps))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = warmstart.train(plan, net, train_steps, seed0=w.seed * 1000, crop=(64, 64, 64), lr=1e-3, lr_final=1e-5,
                           n_spheres=w.n_blobs, n_tubes=w.n_tubes, log=log, log_every=max(1, train_steps // 10))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    # warm the captured solver graphs before timing
    d0 = plan.noisy_data(plan.phantom(1), 1, 30.0, 3.0)
    plan.solve(d0, max_iter=20, tol=0.0, tau=0.0)
    net.warm_start(plan, d0)
    torch.cuda.synchronize()
    res = warmstart.compare(plan, net, [w.seed * 1000 + 10_000_000 + j for j in range(n_eval)], tol=tol,
                            max_iter=max_iter, n_spheres=w.n_blobs, n_tubes=w.n_tubes)
    out = {"workload": w.name, "network_params": net.nparam, "train_steps": train_steps,
           "train_s": round(train_s, 2), "train_ms_per_step": round(1e3 * train_s / max(1, train_steps), 3),
           "loss_first_last": [hist[0][1], hist[-1][1]], "eval_samples": n_eval,
           "cold_iters": [r["cold_iters"] for r in res], "warm_iters": [r["warm_iters"] for r in res],
           "cold_s": [round(r["cold_s"], 4) for r in res], "warm_s": [round(r["warm_s"], 4) for r in res]}
    out["iters_ratio"] = round(float(np.sum(out["warm_iters"]) / np.sum(out["cold_iters"])), 4)
    out["speedup"] = round(float(np.sum(out["cold_s"]) / np.sum(out["warm_s"])), 4)
    out["warm_vs_cold_rel_l2"] = [round(float((r["warm"] - r["cold"]).norm() / r["cold"].norm()), 5) for r in res]
    out["truth_rel_l2_cold_warm_init"] = [
        [round(float((r[k] - r["truth"]).norm() / r["truth"].norm()), 5) for k in ("cold", "warm", "init")]
        for r in res]
    return out


SHIPPED_TILES = os.path.join(ROOT, "paper_2503_13802_amd", "tiles_gfx950.json")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_class_workload1.md")


def vector_leg(w, steps, warmup, tile_cache=None):
    """The vector model (eq. matrixModel) on the workload's grid: seeded synthetic
    component PSFs and sensitivities for C = 1 (user spectra, complex) and C = 3;
    fused A+A^T applications per second and the class passes' HBM rate."""
    import torch
    from paper_2503_13802_amd import inputs, mh3d
    dev = torch.device("cuda:0")
    K = len(w.harmonics)
    out = {"grid": list(w.shape), "harmonics": list(w.harmonics), "decimation": list(w.ds),
           "inputs": "inputs.vector_psfs / vector_sensitivity (seeded synthetic)"}
    rho = torch.tensor(inputs.phantom(w), dtype=torch.float32, device=dev)
    for C in (1, 3):
        h = inputs.vector_psfs(C, K, w.shape, 7000 + C)
        b = inputs.vector_sensitivity(C, w.shape, 7100 + C)
        if C == 1:
            h, b = h[0], b[0]
        plan = mh3d.Plan(w.shape, w.harmonics, 1.0, w.ds, 1.0, w.lam, psf=torch.tensor(h, dtype=torch.float32),
                         sens=torch.tensor(b, dtype=torch.float32))
        tiles = plan.tiles()
        if tile_cache is not None:
            tiles, _ = plan.autotune(tile_cache)
        y = torch.empty((K,) + w.small_shape, device=dev)
        x = torch.empty(w.shape, device=dev)
        for _ in range(warmup):
            plan.forward_adjoint(rho, d_out=y, x_out=x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.forward_adjoint(rho, d_out=y, x_out=x)
        torch.cuda.synchronize()
        rate = steps / (time.perf_counter() - t0)
        pass_us = plan.time_passes(reps=100)
        kern, spec, avg_s = class_roofline(pass_us, w, compact=False, ncomp=C)
        out["C%d" % C] = {"applications_per_s": round(rate, 2), "tiles": list(tiles),
                          "kernels_us": {k: round(v, 3) for k, v in pass_us.items()},
                          "class_kernel": kern.split(" ")[0],
                          "class_bytes_per_launch": spec, "class_GBps": round(spec / avg_s / 1e9, 1)}
        log("vector C=%d: %.1f A+A^T/s, tiles %s" % (C, rate, tiles))
        plan.close()
    out["C3_over_C1_time"] = round(out["C1"]["applications_per_s"] / out["C3"]["applications_per_s"], 3)
    return out


def mh2d_leg(steps, warmup, tile_cache=None):
    """The 2D projection geometry (Sec. 5.2): a 128 x 256 image, two scans (drive along
    x, then z), k = 2..8 each, stacked as the vector model with one PSF block per
    harmonic; seeded synthetic scan PSFs and sensitivities, spiral phantom, 30 dB noise.
    Fused A+A^T applications per second and the time to reconstruct at r_k <= 1e-4."""
    import numpy as np
    import torch
    from paper_2503_13802_amd import inputs, mh3d
    dev = torch.device("cuda:0")
    w = inputs.mh2d_workload()
    K = len(w.harmonics)
    hs = [inputs.scan_psfs(K, w.shape, ax, w.seed + ax) for ax in w.drive_axes]
    bs = [inputs.vector_sensitivity(1, w.shape, w.seed + 10 + ax)[0] for ax in w.drive_axes]
    psf, sens = mh3d.stack_scans(hs, bs)
    plan = mh3d.Plan(w.shape, w.harmonics * len(hs), 1.0, w.ds, 1.0, w.lam, psf=torch.tensor(psf, device=dev),
                     sens=torch.tensor(sens, device=dev))
    tiles = plan.tiles()
    if tile_cache is not None:
        tiles, _ = plan.autotune(tile_cache)
    rho = torch.tensor(inputs.spiral_phantom_2d(w), dtype=torch.float32, device=dev)
    clean = plan.forward(rho).cpu().numpy().astype(np.float64)
    xi = inputs.noise_draw(w, n_harm=clean.shape[0])
    d = torch.tensor(inputs.add_noise(clean, [w.snr_db] * clean.shape[0], xi), dtype=torch.float32, device=dev)
    y = torch.empty_like(d)
    x = torch.empty_like(rho)
    for _ in range(warmup):
        plan.forward_adjoint(rho, d_out=y, x_out=x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.forward_adjoint(rho, d_out=y, x_out=x)
    torch.cuda.synchronize()
    rate = steps / (time.perf_counter() - t0)
    rho_init = torch.zeros_like(rho)   # the start image, resident before the clock starts
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rec, info = plan.solve(d, rho0=rho_init, max_iter=w.max_iter, tol=w.tol, tau=0.0)
    torch.cuda.synchronize()
    first_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    rec2, info2 = plan.solve(d, rho0=rho_init, max_iter=w.max_iter, tol=w.tol, tau=0.0)
    torch.cuda.synchronize()
    cached_s = time.perf_counter() - t0
    out = {"workload": w.name, "grid": list(w.shape), "scans": len(hs), "harmonics_per_scan": list(w.harmonics),
           "decimation": list(w.ds), "lambda": w.lam, "tiles": list(tiles),
           "inputs": "inputs.scan_psfs / vector_sensitivity / spiral_phantom_2d (seeded synthetic)",
           "applications_per_s": round(rate, 2),
           "kernels_us": {k: round(v, 3) for k, v in plan.time_passes(reps=100).items()},
           "time_to_recon": {"plain_s": round(first_s, 4), "plain_cached_step_s": round(cached_s, 4),
                             "iters": info["iters"], "rel_step": info["rel_step"],
                             "ms_per_iter": round(info2["ms_per_iter"], 4), "status": info["status"],
                             "identical_rerun": bool(torch.equal(rec, rec2))}}
    log("mh2d: %.1f A+A^T/s, solve %d updates in %.3f s" % (rate, info["iters"], first_s))
    plan.close()
    return out


def tile_cache_path(arg):
    """The autotuner cache: the given path, else a temp copy of the shipped one."""
    if arg:
        return arg
    import shutil
    import tempfile
    path = os.path.join(tempfile.gettempdir(), "mh3d_tiles.json")
    if os.path.exists(SHIPPED_TILES) and not os.path.exists(path):
        shutil.copyfile(SHIPPED_TILES, path)
    return path


def kernel_source_hash():
    """Hash of the HIP sources; counter results are only valid for the code they measured."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2503_13802_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def stored_traffic(workload_name, tiles, kernel):
    """HBM bytes per launch of the named class kernel from the committed counter
    summary, if it was taken on the current kernel sources, workload and tiles (else
    None)."""
    try:
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if line.startswith("traffic-json: "):
                    t = json.loads(line[len("traffic-json: "):])
                    if (t["source_hash"] == kernel_source_hash() and t["workload"] == workload_name
                            and list(t["tiles"]) == list(tiles) and t["kernel"] == kernel):
                        return t
    except (OSError, ValueError, KeyError):
        pass
    return None


def pmc_driver(args):
    """Counter-run driver: tuned plan of the workload, 20 A+A^T steps as the bench times
    them (three launches, the fused class pass) and 20 as separate forward and adjoint
    calls (six launches), then a 256 MiB device copy (the calibration kernel of known size)."""
    import torch
    from paper_2503_13802_amd import inputs, mh3d
    w = inputs.workload(args.workload)
    plan = mh3d.Plan(w.shape, w.harmonics, w.a_per_mm, w.ds, w.sigma_mm, w.lam, w.voxel_mm)
    if not args.no_tune:
        plan.autotune(tile_cache_path(args.tile_cache))
    dev = torch.device("cuda:0")
    src = torch.tensor(inputs.random_field(w.shape, 1), dtype=torch.float32, device=dev)
    y = torch.empty((len(w.harmonics),) + w.small_shape, device=dev)
    x = torch.empty(w.shape, device=dev)
    for _ in range(20):
        plan.forward_adjoint(src, d_out=y, x_out=x)
        plan.forward(src, out=y)
        plan.adjoint(y, out=x)
    a = torch.ones(64 << 20, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print("pmc driver: %s tiles %s, 20 fused and 20 separate A+A^T steps, 5 copies of 256 MiB"
          % (w.name, plan.tiles()), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", type=int, default=1, choices=[1, 2])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-volumes", type=int, default=64)
    ap.add_argument("--no-warm", action="store_true")
    ap.add_argument("--no-vector", action="store_true")
    ap.add_argument("--no-mh2d", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="heuristic tiles instead of the autotuner")
    ap.add_argument("--tile-cache", default=None, help="autotuner JSON cache (default: a file in the temp dir)")
    ap.add_argument("--warm-train-steps", type=int, default=20000)
    ap.add_argument("--warm-eval", type=int, default=4)
    ap.add_argument("--pmc-driver", action="store_true",
                    help="only run the workload's A+A^T steps and a copy of known size (for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only; more GPUs would each take whole volumes of a batch "
              "with no exchange between them, which is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    from paper_2503_13802_amd import inputs

    if args.pmc_driver:
        pmc_driver(args)
        return

    batch_inputs = None
    if not args.no_batch:
        # host phantoms of the batch workload, drawn in worker processes before the
        # GPU is touched
        from multiprocessing import Pool
        bws = inputs.batch_workloads(args.batch_volumes)
        t0 = time.perf_counter()
        with Pool(min(16, os.cpu_count() or 1)) as pool:
            phantoms = pool.map(inputs.phantom, bws)
        batch_inputs = (bws, phantoms, time.perf_counter() - t0)
        log("batch phantoms: %d volumes in %.1f s" % (len(bws), batch_inputs[2]))

    import torch
    from paper_2503_13802_amd import mh3d

    w = inputs.workload(args.workload)
    log("workload %s" % w.name)
    rho_true = inputs.phantom(w)
    xi = inputs.noise_draw(w)
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    plan = mh3d.Plan(w.shape, w.harmonics, w.a_per_mm, w.ds, w.sigma_mm, w.lam, w.voxel_mm)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    tile_cache = None
    tuning = {"heuristic_tiles": list(plan.tiles())}
    if not args.no_tune:
        tile_cache = tile_cache_path(args.tile_cache)
        t0 = time.perf_counter()
        tiles, us = plan.autotune(tile_cache)
        tuning.update({"tiles": list(tiles), "tuned_us_per_application": round(us, 3),
                       "tune_s": round(time.perf_counter() - t0, 3)})
        log("autotuned tiles %s (%.2f us per A+A^T)" % (tiles, us))
    rho_t = torch.tensor(rho_true, dtype=torch.float32, device=dev)
    clean = plan.forward(rho_t).cpu().numpy().astype(np.float64)
    d = torch.tensor(inputs.add_noise(clean, w.snr_db, xi), dtype=torch.float32, device=dev)
    x = torch.empty(w.shape, device=dev)
    y = torch.empty((len(w.harmonics),) + w.small_shape, device=dev)
    src = rho_t.clone()

    def step():
        # d = A src and x = A^T d (three launches: A^T starts from d's decimated spectra)
        plan.forward_adjoint(src, d_out=y, x_out=x)

    def step_separate():
        plan.forward(src, out=y)
        plan.adjoint(y, out=x)

    for _ in range(args.warmup):
        step()
        step_separate()
    torch.cuda.synchronize()
    log("timing %d steps" % args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    value = args.steps / wall
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step_separate()
    torch.cuda.synchronize()
    separate_per_s = args.steps / (time.perf_counter() - t0)

    # per-kernel HIP-event timing over a second pass of the same steps
    plan.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall_prof = time.perf_counter() - t0
    prof = plan.profile_read()
    plan.profile(False)
    op_bytes = algorithmic_bytes(w)[0]
    # the dominant kernel's launch duration: back-to-back launches between two HIP
    # events on the plan's stream (per-launch events would add their own overhead)
    pass_us = plan.time_passes(reps=200)
    kern, spec_bytes, avg_s = class_roofline(pass_us, w)
    achieved = spec_bytes / avg_s / 1e9
    kernels = {k: {"avg_us": 1e3 * v[0] / v[1], "launches": v[1]} for k, v in prof.items() if v[1]}
    st = stored_traffic(w.name, plan.tiles(), kern.split(" ")[0])
    traffic = None if st is None else st["bytes_per_launch"]
    log("kernels: " + json.dumps(kernels))

    out = {
        "metric": "A+A^T applications/s & time-to-recon at rel.residual 1e-4 (plain vs warm/batched)",
        "value": round(value, 2),
        "unit": "A+A^T applications/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": list(w.shape), "harmonics": list(w.harmonics),
                   "decimation": list(w.ds), "a_per_mm": w.a_per_mm, "lambda": w.lam},
        "roofline": {"bound": "hbm", "kernel": kern,
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "bytes_per_launch": spec_bytes, "avg_launch_us": round(avg_s * 1e6, 3)},
        "separate_calls_per_s": round(separate_per_s, 2),
        "operator_GBps": round(2 * op_bytes / (ms_per_step / 1e3) / 1e9, 1),
        "operator_bytes_per_application": op_bytes,
        "kernels_us": {k: round(v, 3) for k, v in pass_us.items()},
        "kernels_us_event_per_launch": {k: round(v["avg_us"], 3) for k, v in kernels.items()},
        "ms_per_step_profiled": round(1e3 * wall_prof / args.steps, 4),
        "plan_s": round(plan_s, 3),
        "tiles": tuning,
    }

    if not args.no_solve:
        log("plain solve to r <= %g" % w.tol)
        # the start image rho = 0 is an input of the solve: resident before the clock starts
        rho_init = torch.zeros(w.shape, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec, info = plan.solve(d, rho0=rho_init, max_iter=w.max_iter, tol=w.tol, tau=0.0, power_iters=50,
                               power_seed=0)
        torch.cuda.synchronize()
        first_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        rec2, info2 = plan.solve(d, rho0=rho_init, max_iter=w.max_iter, tol=w.tol, tau=0.0, power_iters=50,
                                 power_seed=0)
        torch.cuda.synchronize()
        out["time_to_recon"] = {"plain_s": round(first_s, 4), "plain_cached_step_s": round(time.perf_counter() - t0, 4),
                                "iters": info["iters"], "rel_step": info["rel_step"],
                                "ms_per_iter": round(info2["ms_per_iter"], 4), "tau": info["tau"],
                                "status": info["status"], "identical_rerun": bool(torch.equal(rec, rec2))}

    if not args.no_vector:
        out["vector_model"] = vector_leg(w, min(args.steps, 200), min(args.warmup, 20), tile_cache)

    if not args.no_mh2d:
        out["mh2d"] = mh2d_leg(min(args.steps, 200), min(args.warmup, 20), tile_cache)

    if batch_inputs is not None:
        out["batched"] = batched_leg(batch_inputs, w.tol, w.max_iter, tile_cache)

    if not args.no_warm:
        out["warm_start"] = warm_leg(args.warm_train_steps, args.warm_eval, w.tol, w.max_iter,
                                     tile_cache=tile_cache)

    if not args.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w, rho_true, xi, plan=None if args.no_solve else plan)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
