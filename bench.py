"""Benchmark of the MH3D hot path on one MI355X.

The headline workload is the 128^3 grid with harmonics k = 2..12 and decimation (2, 4, 4)
(the largest single-GPU workload).  A step is one application of the forward operator A
followed by its adjoint A^T applied to A's output (Sec. 4.1 eq. dN; each accelerated
projected-gradient update of Sec. 4.3 costs one of each) on resident inputs: d = A rho is
written to HBM and x = A^T d is computed, in three launches (forward plane pass, column
pass, adjoint plane pass beside the small-grid pass that writes d).  `value` is that
fused rate; the rate of A and A^T as two separate calls on independent inputs (the
adjoint starting from portraits in HBM) is reported beside it.

The JSON line also reports the HBM roofline of the dominant kernel (algorithmic bytes per
launch over its duration, measured with HIP events around back-to-back launches on the
plan's stream; HBM traffic from the committed rocprofv3 counter summary when it was taken
on the current kernel sources), the FP64-oracle relative L2 error of every reported result,
the time to reconstruct at r_k <= 1e-4 (plain; batched; warm-started), and the FP64 CPU
oracle timed on the host cores.

Oracle work runs in a CPU process started before the GPU is touched (the oracle's data
for the 128^3 and 96x96x64 reconstructions, its step sizes and its FISTA runs) and is
joined before the CPU baseline is timed, so the baseline runs on an idle host.

Legs (each can be skipped): secondary workload 96x96x64 k = 2..8; the vector model of eq.
matrixModel (C = 1 and 3) and the MH2D projection geometry of Sec. 5.2 (rates and oracle
errors); the batch of 64 uneven volumes (sequential vs batched solves, setup included);
the learned warm start (GPU training on 20k generated pairs, then cold vs warm solves on
32 held-out samples with the FP64 oracle's objective at both end points).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 2|1] [--no-cpu]
                       [--no-solve] [--no-secondary] [--no-batch] [--no-warm] [--no-vector]
                       [--no-mh2d] [--warm-train-steps T] [--warm-eval E]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SHIPPED_TILES = os.path.join(ROOT, "paper_2503_13802_amd", "tiles_gfx950.json")
PROFILES = os.path.join(ROOT, "profiles")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def rel_l2(a, b):
    import numpy as np
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ----------------------------------------------------------------------------- bytes
def shape_terms(w):
    nx, ny, nz = w.shape
    mx, my, mz = w.small_shape
    K = len(w.harmonics)
    return dict(nx=nx, ny=ny, nz=nz, mx=mx, my=my, mz=mz, K=K, N=nx * ny * nz, M=mx * my * mz,
                Nc=nx * ny * (nz // 2 + 1), Mc=mx * my * (mz // 2 + 1), ncls=my * (mz // 2 + 1), nzh=nz // 2 + 1,
                sx=w.ds[0], sy=w.ds[1], sz=w.ds[2])


def fast_kernel_bytes(w):
    """Algorithmic bytes per launch of the compile-time (separable) passes of A then A^T:
      plane_fwd      rho, b (8N) + the folded shares written (8 sy nx ncls) + the y-residue
                     table (8 sy my (nz/2+1))
      class_normal   (the column pass) shares read (8 sy nx ncls) + Q written (8 nx ncls)
                     + the decimated spectra G written (8 K mx ncls) + x factors (4 K nx)
      adj_and_store  Q read (8 nx ncls) + table + b read and x written (8N) + G read
                     (8 K mx ncls) + d written (4 K M)
    ncls = my (mz/2 + 1) columns of the folded (y', z') half spectrum."""
    t = shape_terms(w)
    tab = 8 * t["sy"] * t["my"] * t["nzh"]
    share = 8 * t["sy"] * t["nx"] * t["ncls"]
    q = 8 * t["nx"] * t["ncls"]
    g = 8 * t["K"] * t["mx"] * t["ncls"]
    return {"plane_fwd": 8 * t["N"] + share + tab,
            "class_normal": share + q + g + 4 * t["K"] * t["nx"],
            "adj_and_store": q + tab + 8 * t["N"] + g + 4 * t["K"] * t["M"]}


def general_kernel_bytes(w, compact=True, ncomp=1):
    """Algorithmic bytes per launch of the general passes (kernels.hpp): spectra of
    beta_H = 4 (compact) or 8 bytes per element in the class layout."""
    t = shape_terms(w)
    bh = 4 if compact else 8
    C = ncomp
    return {"plane_fwd": 4 * C * t["N"] + 4 * t["N"] + 8 * C * t["Nc"],
            "class_normal": bh * C * t["K"] * t["Nc"] + 16 * C * t["Nc"] + 8 * t["K"] * t["Mc"],
            "adj_and_store": 8 * C * t["Nc"] + 8 * t["N"] + 8 * t["K"] * t["Mc"] + 4 * t["K"] * t["M"],
            "class_fwd": bh * C * t["K"] * t["Nc"] + 8 * C * t["Nc"] + 8 * t["K"] * t["Mc"],
            "class_adj": bh * C * t["K"] * t["Nc"] + 8 * C * t["Nc"] + 8 * t["K"] * t["Mc"]}


def operator_bytes(w, separable=True, ncomp=1):
    """Algorithmic bytes of one application of A (A^T moves the same): rho (4N), the
    sensitivities (4CN), the PSF data (separable: the x factors and the y-residue table;
    else beta_H C K N_c spectra) and the portraits (4KM)."""
    t = shape_terms(w)
    if separable:
        spectra = 4 * t["K"] * t["nx"] + 8 * t["sy"] * t["my"] * t["nzh"]
    else:
        spectra = 8 * ncomp * t["K"] * t["Nc"]
    return 4 * t["N"] + 4 * ncomp * t["N"] + spectra + 4 * t["K"] * t["M"]


def roofline(pass_us, byte_map, kernels):
    """The dominant kernel of the step (longest average launch in pass_us: microseconds
    per launch over back-to-back launches of each pass between two HIP events on the
    plan's stream, mh3d_time_pass) with its algorithmic bytes per launch and its average
    launch duration in seconds."""
    name = max(kernels, key=lambda k: pass_us[k])
    s = pass_us[name] * 1e-6
    return name, byte_map[name], s


# ----------------------------------------------------------------------------- traffic
def kernel_source_hash():
    """Hash of the HIP sources; counter results are only valid for the code they measured."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2503_13802_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def stored_traffic(workload_name, kernel):
    """HBM bytes per launch of the named kernel from a committed counter summary
    (profiles/traffic_*.md, line 'traffic-json: ...'), if it was taken on the current
    kernel sources and workload (else None)."""
    try:
        names = sorted(n for n in os.listdir(PROFILES) if n.startswith("traffic_") and n.endswith(".md"))
    except OSError:
        return None
    for n in names:
        try:
            with open(os.path.join(PROFILES, n)) as f:
                for line in f:
                    if line.startswith("traffic-json: "):
                        t = json.loads(line[len("traffic-json: "):])
                        if t["source_hash"] == kernel_source_hash() and t["workload"] == workload_name:
                            b = t["per_launch_bytes"].get(kernel)
                            if b is not None:
                                return int(b)
        except (OSError, ValueError, KeyError):
            continue
    return None


# ----------------------------------------------------------------------------- oracle process
def oracle_jobs(wl_ids, q, workers):
    """CPU process: for each workload the oracle's data (phantom through the FP64 operator
    plus the workload's noise), its step size (50 power iterations from the Philox start)
    and its FISTA reconstruction to r_k <= tol; results go to q as they are ready."""
    import numpy as np
    from oracle import model as om
    from oracle import philox as oph
    from oracle import solver as osv
    from paper_2503_13802_amd import inputs
    om._workers = lambda: workers   # leave host cores to the GPU driver process
    for wl in wl_ids:
        w = inputs.workload(wl)
        h = om.psf_bank(w.shape, list(w.harmonics), w.a_per_mm, w.voxel_mm)
        b = om.sensitivity(w.shape, w.sigma_mm, w.voxel_mm)
        op = osv.Operator(h, b, w.ds, w.lam)
        rho = inputs.phantom(w)
        d = inputs.add_noise(op.A(rho), w.snr_db, inputs.noise_draw(w))
        q.put(("data", wl, d.astype(np.float32)))
        t0 = time.perf_counter()
        tau = osv.step_size(osv.power_iteration(op, oph.uniform01(0, 0, w.n_voxels).reshape(w.shape), 50))
        q.put(("tau", wl, tau))
        rec, _, n = osv.fista(op, d, tau, max_iter=w.max_iter, tol=w.tol)
        q.put(("recon", wl, (rec, n, time.perf_counter() - t0)))
    q.put(("done", None, None))


class OracleResults:
    def __init__(self, q, proc):
        self.q, self.proc, self.got = q, proc, {}
        self.paused = 0

    def pause(self):
        """Stop the oracle process (SIGSTOP) while the GPU is timed: its FFT threads would
        otherwise slow the host thread that launches the kernels."""
        import signal
        if self.paused == 0 and self.proc.is_alive():
            os.kill(self.proc.pid, signal.SIGSTOP)
        self.paused += 1

    def resume(self):
        import signal
        self.paused -= 1
        if self.paused == 0 and self.proc.is_alive():
            os.kill(self.proc.pid, signal.SIGCONT)

    def get(self, kind, wl, timeout=900):
        import queue
        assert self.paused == 0
        while (kind, wl) not in self.got:
            try:
                k, w, v = self.q.get(timeout=timeout)
            except queue.Empty:
                raise RuntimeError("oracle process gave no %s for workload %s" % (kind, wl))
            self.got[(k, w)] = v
        return self.got[(kind, wl)]

    def join(self):
        self.get("done", None)
        self.proc.join(timeout=60)


class Quiet:
    """Context of a timed GPU section: the oracle process (if any) is paused."""
    oracle = None

    def __enter__(self):
        if Quiet.oracle is not None:
            Quiet.oracle.pause()

    def __exit__(self, *a):
        if Quiet.oracle is not None:
            Quiet.oracle.resume()


# ----------------------------------------------------------------------------- CPU baseline
def cpu_info():
    import numpy as np
    import scipy
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "numpy": np.__version__, "scipy": scipy.__version__}


def cpu_baseline(w, rho, r, budget_s=12.0):
    """The FP64 oracle as it stands, timed on the host cores: full A+A^T applications of
    the FFT tier (scipy.fft, workers = all cores) until the budget is spent; the same on
    one core (a bounded number); and the direct-sum tier (the definition, eq. dN) timed on
    a random sample of output entries of A and voxels of A^T and extrapolated to a whole
    application."""
    import numpy as np
    from oracle import model as om
    h = om.psf_bank(w.shape, list(w.harmonics), w.a_per_mm, w.voxel_mm)
    b = om.sensitivity(w.shape, w.sigma_mm, w.voxel_mm)
    n = 0
    t0 = time.perf_counter()
    while True:
        om.forward_fft(h, b, rho, w.ds)
        om.adjoint_fft(h, b, r, w.ds)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 50:
            break
    rate = n / el
    t0 = time.perf_counter()
    om.forward_fft(h, b, rho, w.ds, workers=1)
    om.adjoint_fft(h, b, r, w.ds, workers=1)
    single = 1.0 / (time.perf_counter() - t0)
    rng = np.random.default_rng(7)
    ne = 32
    ent = [(int(rng.integers(len(w.harmonics))),) + tuple(int(rng.integers(m)) for m in w.small_shape)
           for _ in range(ne)]
    vox = [tuple(int(rng.integers(m)) for m in w.shape) for _ in range(ne)]
    t0 = time.perf_counter()
    om.forward_direct_at(h, b, rho, w.ds, ent)
    ta = (time.perf_counter() - t0) / ne
    t0 = time.perf_counter()
    om.adjoint_direct_at(h, b, r, w.ds, vox)
    tt = (time.perf_counter() - t0) / ne
    n_out = len(w.harmonics) * int(np.prod(w.small_shape))
    n_vox = int(np.prod(w.shape))
    direct = 1.0 / (ta * n_out + tt * n_vox)
    out = {"value": rate, "unit": "A+A^T applications/s", "cores": os.cpu_count(), "kind": "oracle",
           "sample": "%d full A+A^T applications of the FP64 FFT-tier oracle (scipy.fft, workers=%d) on the "
                     "headline workload, %.1f s" % (n, os.cpu_count(), el),
           "single_core_per_s": single,
           "direct_sum_per_s_extrapolated": direct,
           "direct_sum_sample": "%d entries of A (%.2f ms each) and %d voxels of A^T (%.2f ms each) by direct "
                                "sums, extrapolated to %d entries and %d voxels (single-threaded NumPy)"
                                % (ne, 1e3 * ta, ne, 1e3 * tt, n_out, n_vox)}
    out.update(cpu_info())
    return out


# ----------------------------------------------------------------------------- GPU legs
def time_steps(fn, steps, warmup, repeats=1):
    """Seconds per step over `steps` steps after `warmup` untimed ones; with repeats > 1
    the median of that many such loops (the secondary legs, one short loop of which can
    catch a transient of the host or the GPU)."""
    import torch
    with Quiet():
        for _ in range(warmup):
            fn()
        times = []
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                fn()
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) / steps)
        return sorted(times)[len(times) // 2]


def operator_leg(w, steps, warmup, tile_cache, oracle_check=True, repeats=1):
    """Fused A then A^T rate, separate-call rate, per-pass durations, roofline of the
    dominant kernel, and the FP64-oracle error of A and A^T on the phantom."""
    import numpy as np
    import torch
    from paper_2503_13802_amd import inputs, mh3d
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    plan = mh3d.Plan(w.shape, w.harmonics, w.a_per_mm, w.ds, w.sigma_mm, w.lam, w.voxel_mm)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    tuning = {"heuristic_tiles": list(plan.tiles())}
    if tile_cache is not None:
        tiles, us = plan.autotune(tile_cache)
        tuning.update({"tiles": list(tiles), "tuned_us_per_application": round(us, 3)})
    separable = plan.path() == 1
    rho = inputs.phantom(w)
    src = torch.tensor(rho, dtype=torch.float32, device=dev)
    K = len(w.harmonics)
    y = torch.empty((K,) + w.small_shape, device=dev)
    x = torch.empty(w.shape, device=dev)
    r = torch.tensor(inputs.noise_draw(w), dtype=torch.float32, device=dev)
    x2 = torch.empty(w.shape, device=dev)
    y2 = torch.empty((K,) + w.small_shape, device=dev)

    def fused():
        plan.forward_adjoint(src, d_out=y, x_out=x)

    def separate():   # A on rho, A^T on independent portraits
        plan.forward(src, out=y2)
        plan.adjoint(r, out=x2)

    sec = time_steps(fused, steps, warmup, repeats)
    # per-launch durations in steps like the timed ones: the same steps again with HIP
    # events around every launch on the plan's stream (mh3d_profile); each event pair
    # adds its own wait to the launch it brackets, so these read above the kernels
    with Quiet():
        plan.profile(True)
        for _ in range(steps):
            fused()
        prof = plan.profile_read()
        plan.profile(False)
    live_us = {k: 1e3 * ms / n for k, (ms, n) in prof.items() if n}
    sec_sep = time_steps(separate, steps, warmup, repeats)
    with Quiet():
        pass_us = plan.time_passes(reps=200)
    byte_map = fast_kernel_bytes(w) if separable else general_kernel_bytes(w)
    kern, kbytes, ks = roofline(pass_us, byte_map, ["plane_fwd", "class_normal", "adj_and_store"])
    achieved = kbytes / ks / 1e9
    op_b = operator_bytes(w, separable)
    out = {"rate": 1.0 / sec, "ms_per_step": 1e3 * sec, "separate_rate": 1.0 / sec_sep,
           "roofline": {"bound": "hbm", "kernel": kern, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": stored_traffic(w.name, kern),
                        "bytes_per_launch": kbytes, "avg_launch_us": round(ks * 1e6, 3)},
           "kernels_us_in_step": {k: round(v, 3) for k, v in live_us.items()},
           "kernels_us": {k: round(v, 3) for k, v in pass_us.items()},
           "kernel_bytes_per_launch": byte_map,
           "operator_bytes_per_application": op_b,
           "operator_GBps": round(2 * op_b / sec / 1e9, 1),
           "path": "compile-time separable passes" if separable else "general passes",
           "plan_s": round(plan_s, 3), "tiles": tuning}
    if oracle_check:
        from oracle import model as om
        h = om.psf_bank(w.shape, list(w.harmonics), w.a_per_mm, w.voxel_mm)
        b = om.sensitivity(w.shape, w.sigma_mm, w.voxel_mm)
        d_ref = om.forward_fft(h, b, rho, w.ds)
        rn = r.cpu().numpy().astype(np.float64)
        out["oracle_rel_l2"] = {"A_fused": rel_l2(y.cpu().numpy(), d_ref),
                                "AT_fused": rel_l2(x.cpu().numpy(), om.adjoint_fft(h, b, d_ref, w.ds)),
                                "A_separate": rel_l2(y2.cpu().numpy(), d_ref),
                                "AT_separate": rel_l2(x2.cpu().numpy(), om.adjoint_fft(h, b, rn, w.ds)),
                                "reference": "FP64 FFT-tier oracle (pinned to the direct sums) on the same inputs"}
    return plan, out


def solve_leg(plan, w, oracle, wl):
    """Time to reconstruct at r_k <= tol from rho = 0 on the oracle's data (resident
    before the clock): first call (power iteration for tau included) and repeated call
    (tau cached).  Returns (result dict, data tensor) for solve_check."""
    import torch
    dev = torch.device("cuda:0")
    d = torch.tensor(oracle.get("data", wl), device=dev)
    rho0 = torch.zeros(w.shape, device=dev)
    with Quiet():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec, info = plan.solve(d, rho0=rho0, max_iter=w.max_iter, tol=w.tol, tau=0.0, power_iters=50, power_seed=0)
        torch.cuda.synchronize()
        first_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        rec2, info2 = plan.solve(d, rho0=rho0, max_iter=w.max_iter, tol=w.tol, tau=0.0, power_iters=50, power_seed=0)
        torch.cuda.synchronize()
        cached_s = time.perf_counter() - t0
    out = {"plain_s": round(first_s, 4), "plain_cached_tau_s": round(cached_s, 4), "iters": info["iters"],
           "rel_step": info["rel_step"], "ms_per_iter": round(info2["ms_per_iter"], 4), "tau": info["tau"],
           "status": info["status"], "identical_rerun": bool(torch.equal(rec, rec2))}
    return out, d


def solve_check(plan, w, oracle, wl, d):
    """At the oracle's tau and its update count, the relative L2 difference of the GPU
    reconstruction from the oracle's (both from rho = 0 on the oracle's data), and the GPU's
    own update count to r_k <= tol at that tau."""
    import torch
    rho0 = torch.zeros(w.shape, device=d.device)
    tau_o = oracle.get("tau", wl)
    want, n_o, o_s = oracle.get("recon", wl)
    got, _ = plan.solve(d, rho0=rho0, max_iter=n_o, tol=0.0, tau=tau_o)
    _, gi_tol = plan.solve(d, rho0=rho0, max_iter=w.max_iter, tol=w.tol, tau=tau_o)
    return {"oracle_rel_l2": rel_l2(got.cpu().numpy(), want), "oracle_iters": int(n_o),
            "gpu_iters_at_oracle_tau": gi_tol["iters"], "oracle_tau": tau_o, "oracle_solve_s": round(o_s, 2),
            "note": "oracle-made data (phantom through the FP64 operator plus the workload's noise); the GPU runs "
                    "the oracle's update count at the oracle's step size"}


def vector_leg(w, steps, warmup, tile_cache=None):
    """The vector model (eq. matrixModel) on the workload's grid: seeded synthetic
    component PSFs and sensitivities for C = 1 (user spectra, complex) and C = 3; fused
    A+A^T rate, the class passes' HBM rate and the FP64-oracle error of A and A^T."""
    import numpy as np
    import torch
    from oracle import model as om
    from paper_2503_13802_amd import inputs, mh3d
    dev = torch.device("cuda:0")
    K = len(w.harmonics)
    out = {"grid": list(w.shape), "harmonics": list(w.harmonics), "decimation": list(w.ds),
           "inputs": "inputs.vector_psfs / vector_sensitivity (seeded synthetic)"}
    rho = inputs.phantom(w)
    src = torch.tensor(rho, dtype=torch.float32, device=dev)
    for C in (1, 3):
        h = inputs.vector_psfs(C, K, w.shape, 7000 + C)
        b = inputs.vector_sensitivity(C, w.shape, 7100 + C)
        if C == 1:
            hp, bp = h[0], b[0]
        else:
            hp, bp = h, b
        plan = mh3d.Plan(w.shape, w.harmonics, 1.0, w.ds, 1.0, w.lam, psf=torch.tensor(hp, dtype=torch.float32),
                         sens=torch.tensor(bp, dtype=torch.float32))
        tiles = plan.tiles()
        if tile_cache is not None:
            tiles, _ = plan.autotune(tile_cache)
        y = torch.empty((K,) + w.small_shape, device=dev)
        x = torch.empty(w.shape, device=dev)
        sec = time_steps(lambda: plan.forward_adjoint(src, d_out=y, x_out=x), steps, warmup, repeats=3)
        pass_us = plan.time_passes(reps=100)
        bmap = general_kernel_bytes(w, compact=False, ncomp=C)
        if "class_normal" in pass_us:
            ck, cb, cs = "class_normal", bmap["class_normal"], pass_us["class_normal"]
        else:
            ck, cb, cs = "class_fwd+class_adj", bmap["class_fwd"], 0.5 * (pass_us["class_fwd"] + pass_us["class_adj"])
        d_ref = om.forward_vector(h, b, rho, w.ds)
        out["C%d" % C] = {"applications_per_s": round(1.0 / sec, 2), "timing": "median of 3 loops of the steps",
                          "tiles": list(tiles),
                          "kernels_us": {k: round(v, 3) for k, v in pass_us.items()},
                          "class_kernel": ck, "class_bytes_per_launch": cb, "class_GBps": round(cb / cs / 1e3, 1),
                          "oracle_rel_l2": {"A": rel_l2(y.cpu().numpy(), d_ref),
                                            "AT": rel_l2(x.cpu().numpy(), om.adjoint_vector(h, b, d_ref, w.ds))}}
        log("vector C=%d: %.1f A+A^T/s" % (C, 1.0 / sec))
        plan.close()
    out["C3_over_C1_time"] = round(out["C1"]["applications_per_s"] / out["C3"]["applications_per_s"], 3)
    return out


def mh2d_leg(steps, warmup, tile_cache=None):
    """The 2D projection geometry (Sec. 5.2): a 128 x 256 image, two scans (drive along x,
    then z), k = 2..8 each, stacked as the vector model; seeded synthetic scan PSFs and
    sensitivities, spiral phantom, 30 dB noise on oracle-made data.  Fused A+A^T rate,
    time to reconstruct at r_k <= 1e-4, and the FP64-oracle errors of A, A^T and the
    reconstruction (at the oracle's step size and update count)."""
    import numpy as np
    import torch
    from oracle import model as om
    from oracle import solver as osv
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
    rho = inputs.spiral_phantom_2d(w)
    h_o, b_o = om.stack_scans([np.asarray(h, np.float64) for h in hs], [np.asarray(b, np.float64) for b in bs])
    op = osv.Operator(h_o, b_o, w.ds, w.lam)
    clean = op.A(rho)
    xi = inputs.noise_draw(w, n_harm=clean.shape[0])
    d_np = inputs.add_noise(clean, [w.snr_db] * clean.shape[0], xi)
    d = torch.tensor(d_np, dtype=torch.float32, device=dev)
    src = torch.tensor(rho, dtype=torch.float32, device=dev)
    y = torch.empty_like(d)
    x = torch.empty_like(src)
    sec = time_steps(lambda: plan.forward_adjoint(src, d_out=y, x_out=x), steps, warmup, repeats=3)
    a_err = rel_l2(y.cpu().numpy(), clean)
    at_err = rel_l2(x.cpu().numpy(), op.AT(clean))
    rho_init = torch.zeros_like(src)
    with Quiet():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec, info = plan.solve(d, rho0=rho_init, max_iter=w.max_iter, tol=w.tol, tau=0.0)
        torch.cuda.synchronize()
        first_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        rec2, info2 = plan.solve(d, rho0=rho_init, max_iter=w.max_iter, tol=w.tol, tau=0.0)
        torch.cuda.synchronize()
        cached_s = time.perf_counter() - t0
    tau_o = osv.step_size(osv.power_iteration(op, inputs.random_field(w.shape, 5), 100))
    want, _, n_o = osv.fista(op, d_np, tau_o, max_iter=w.max_iter, tol=w.tol)
    got, _ = plan.solve(d, rho0=rho_init, max_iter=n_o, tol=0.0, tau=tau_o)
    out = {"workload": w.name, "grid": list(w.shape), "scans": len(hs), "harmonics_per_scan": list(w.harmonics),
           "decimation": list(w.ds), "lambda": w.lam, "tiles": list(tiles),
           "inputs": "inputs.scan_psfs / vector_sensitivity / spiral_phantom_2d (seeded synthetic)",
           "applications_per_s": round(1.0 / sec, 2), "timing": "median of 3 loops of the steps",
           "kernels_us": {k: round(v, 3) for k, v in plan.time_passes(reps=100).items()},
           "time_to_recon": {"plain_s": round(first_s, 4), "plain_cached_tau_s": round(cached_s, 4),
                             "iters": info["iters"], "rel_step": info["rel_step"],
                             "ms_per_iter": round(info2["ms_per_iter"], 4), "status": info["status"],
                             "identical_rerun": bool(torch.equal(rec, rec2))},
           "oracle_rel_l2": {"A": a_err, "AT": at_err, "reconstruction": rel_l2(got.cpu().numpy(), want),
                             "reconstruction_updates": int(n_o)}}
    log("mh2d: %.1f A+A^T/s, solve %d updates in %.3f s" % (1.0 / sec, info["iters"], first_s))
    plan.close()
    return out


def batched_leg(batch_inputs, tol, max_iter, tile_cache=None):
    """64 uneven volumes to r_k <= tol each: 64 sequential plain solves vs one batched
    solve.  Both forms are timed with their step-size setup (each volume's 50-step power
    iteration: one call per plan sequentially, one batched launch sequence in the batch)
    and without it (tau cached).  Plus a 3-volume batch of one geometry at the FP64
    oracle's step size against the oracle's FISTA on oracle-made data."""
    import numpy as np
    import torch
    from oracle import model as om
    from oracle import solver as osv
    from paper_2503_13802_amd import inputs, mh3d
    bws, phantoms, _ = batch_inputs
    dev = torch.device("cuda:0")

    def build():
        plans, ds = [], []
        for bw, ph in zip(bws, phantoms):
            p = mh3d.Plan(bw.shape, bw.harmonics, bw.a_per_mm, bw.ds, bw.sigma_mm, bw.lam, bw.voxel_mm)
            if tile_cache is not None:
                p.autotune(tile_cache)
            clean = p.forward(torch.tensor(ph, dtype=torch.float32, device=dev)).cpu().numpy().astype(np.float64)
            d = inputs.add_noise(clean, bw.snr_db, inputs.noise_draw(bw))
            plans.append(p)
            ds.append(torch.tensor(d, dtype=torch.float32, device=dev))
        return plans, ds

    plans, ds = build()
    torch.cuda.synchronize()
    # volumes whose own solves run the compile-time passes (batches run the general ones)
    compiled = [p.path() == 1 for p in plans]
    log("batched leg: %d plans built, %d on the compile-time passes" % (len(plans), sum(compiled)))
    batch = mh3d.Batch(plans)
    # warm-up of both forms (graph capture, kernel loading) on a second set of plans, so
    # the timed runs below start with no cached step size
    wplans, wds = build()
    wbatch = mh3d.Batch(wplans)
    wbatch.solve(wds, max_iter=16, tol=0.0, tau=0.0)
    wplans[0].solve(wds[0], max_iter=20, tol=0.0, tau=0.0)
    torch.cuda.synchronize()
    wbatch.close()
    for p in wplans:
        p.close()
    # sequential with setup (each plan's power iteration), then cached
    with Quiet():
        t0 = time.perf_counter()
        seq = [p.solve(d, max_iter=max_iter, tol=tol, tau=0.0) for p, d in zip(plans, ds)]
        torch.cuda.synchronize()
        seq_setup_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        seq = [p.solve(d, max_iter=max_iter, tol=tol, tau=0.0) for p, d in zip(plans, ds)]
        torch.cuda.synchronize()
        seq_s = time.perf_counter() - t0
    # batched with setup: fresh plans (no cached step size), then cached
    plans_b, ds_b = build()
    batch_b = mh3d.Batch(plans_b)
    torch.cuda.synchronize()
    with Quiet():
        t0 = time.perf_counter()
        batch_b.solve(ds_b, max_iter=max_iter, tol=tol, tau=0.0)
        torch.cuda.synchronize()
        bat_setup_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        rhos, infos = batch_b.solve(ds_b, max_iter=max_iter, tol=tol, tau=0.0)
        torch.cuda.synchronize()
        bat_s = time.perf_counter() - t0
    same = all(torch.equal(r, s[0]) for r, s, c in zip(rhos, seq, compiled) if not c)
    maxdiff = max(rel_l2(r.cpu().numpy(), s[0].cpu().numpy()) for r, s in zip(rhos, seq))
    iters_seq = [s[1]["iters"] for s in seq]
    iters_bat = [i["iters"] for i in infos]
    conv = sum(1 for i in infos if i["rel_step"] <= tol)
    vox = sum(int(np.prod(bw.shape)) for bw in bws)
    out = {"volumes": len(plans), "voxels": vox,
           "sequential_s": round(seq_s, 4), "batched_s": round(bat_s, 4), "speedup": round(seq_s / bat_s, 3),
           "sequential_with_setup_s": round(seq_setup_s, 4), "batched_with_setup_s": round(bat_setup_s, 4),
           "speedup_with_setup": round(seq_setup_s / bat_setup_s, 3),
           "converged": conv, "iters_max": max(iters_bat), "iters_mean": round(float(np.mean(iters_bat)), 1),
           "sequential_on_compile_time_passes": sum(compiled),
           "identical_to_sequential_on_general_passes": bool(same), "max_rel_l2_to_sequential": maxdiff,
           "iters_match": iters_seq == iters_bat,
           "note": "setup = each volume's 50-step power iteration for tau (sequential: per plan; batched: one "
                   "batched launch sequence, plus the capture of the batch's graph on its first call); the "
                   "cached runs reuse them"}
    batch_b.close()
    # oracle check: three volumes of one geometry (one operator, so one tau) at the oracle's tau
    sub = [i for i, bw in enumerate(bws) if bw.shape == bws[0].shape and bw.harmonics == bws[0].harmonics][:3]
    bw = bws[sub[0]]
    h = om.psf_bank(bw.shape, list(bw.harmonics), bw.a_per_mm, bw.voxel_mm)
    bmap = om.sensitivity(bw.shape, bw.sigma_mm, bw.voxel_mm)
    op = osv.Operator(h, bmap, bw.ds, bw.lam)
    tau_o = osv.step_size(osv.power_iteration(op, inputs.random_field(bw.shape, 77), 60))
    d_o = [inputs.add_noise(op.A(phantoms[i]), bws[i].snr_db, inputs.noise_draw(bws[i])) for i in sub]
    n_fix = 60
    want = [osv.fista(op, dd, tau_o, max_iter=n_fix)[0] for dd in d_o]
    sp = [mh3d.Plan(bw.shape, bw.harmonics, bw.a_per_mm, bw.ds, bw.sigma_mm, bw.lam, bw.voxel_mm) for _ in sub]
    sb = mh3d.Batch(sp)
    got, _ = sb.solve([torch.tensor(dd, dtype=torch.float32, device=dev) for dd in d_o], max_iter=n_fix, tol=0.0,
                      tau=tau_o)
    out["oracle_rel_l2"] = {"volumes": [list(bw.shape) for _ in sub], "harmonics": list(bw.harmonics),
                            "updates": n_fix, "per_volume": [rel_l2(g.cpu().numpy(), wv) for g, wv in zip(got, want)],
                            "note": "a batch of %d volumes of one geometry on oracle-made data at the oracle's step "
                                    "size, against the oracle's FISTA at the same update count" % len(sub)}
    sb.close()
    for p in plans + plans_b + sp:
        p.close()
    return out


def warm_leg(train_steps, n_eval, tol, max_iter, tile_cache=None, n_val=4, n_tight=8, tight_iters=40000):
    """Warm-start workload: GPU training with a fixed validation set evaluated at the start,
    middle and end; then cold vs warm solves to r_k <= tol on n_eval held-out samples, each
    end point compared with the FP64 oracle's objective and with a tight minimiser (the GPU
    solver run to r_k <= 1e-7)."""
    import numpy as np
    import torch
    from oracle import model as om
    from oracle import solver as osv
    from paper_2503_13802_amd import inputs, mh3d, warmstart
    w = inputs.workload(4)
    plan = mh3d.Plan(w.shape, w.harmonics, w.a_per_mm, w.ds, w.sigma_mm, w.lam, w.voxel_mm)
    if tile_cache is not None:
        plan.autotune(tile_cache)
    net = mh3d.Net(WARM_WIDTHS, in_channels=len(w.harmonics), seed=w.seed)
    log("warm leg: %s, network %d parameters, training %d steps" % (w.name, net.nparam, train_steps))
    val = []
    for j in range(n_val):
        seed = w.seed * 1000 + 20_000_000 + j
        rho = plan.phantom(seed, w.n_blobs, w.n_tubes)
        d = plan.noisy_data(rho, seed, warmstart.sample_snr2(seed), 3.0)
        val.append((plan.backproject(d), rho))
    val_loss = []

    def evaluate(j):
        val_loss.append((j, warmstart.validation_loss(plan, net, val)))
        log("validation loss at step %d: %.4e" % (j, val_loss[-1][1]))

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = warmstart.train(plan, net, train_steps, seed0=w.seed * 1000, crop=(64, 64, 64), lr=1e-3, lr_final=1e-5,
                           n_spheres=w.n_blobs, n_tubes=w.n_tubes, log=log, log_every=max(1, train_steps // 10),
                           evaluate=evaluate, eval_at=(0, train_steps // 2, train_steps))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    # warm the solver and the network before timing
    d0 = plan.noisy_data(plan.phantom(1), 1, 30.0, 3.0)
    plan.solve(d0, max_iter=20, tol=0.0, tau=0.0)
    net.warm_start(plan, d0)
    torch.cuda.synchronize()
    with Quiet():
        res = warmstart.compare(plan, net, [w.seed * 1000 + 10_000_000 + j for j in range(n_eval)], tol=tol,
                                max_iter=max_iter, n_spheres=w.n_blobs, n_tubes=w.n_tubes)
    # FP64 oracle objective 1/2 ||A rho - d||^2 + 1/2 lambda ||T rho||^2 of both end points,
    # and their distance to a tight minimiser
    h = om.psf_bank(w.shape, list(w.harmonics), w.a_per_mm, w.voxel_mm)
    b = om.sensitivity(w.shape, w.sigma_mm, w.voxel_mm)
    op = osv.Operator(h, b, w.ds, w.lam)
    obj_c, obj_w, dist_c, dist_w, tight_it, tight_r = [], [], [], [], [], []
    for i, r in enumerate(res):
        dn = r["d"].cpu().numpy().astype(np.float64)
        obj_c.append(op.objective(r["cold"].cpu().numpy().astype(np.float64), dn))
        obj_w.append(op.objective(r["warm"].cpu().numpy().astype(np.float64), dn))
        if i < n_tight:
            tight, ti = plan.solve(r["d"], rho0=r["cold"], max_iter=tight_iters, tol=1e-7, tau=0.0)
            tight_it.append(ti["iters"])
            tight_r.append(ti["rel_step"])
            dist_c.append(float((r["cold"] - tight).norm() / tight.norm()))
            dist_w.append(float((r["warm"] - tight).norm() / tight.norm()))
    ci = [r["cold_iters"] for r in res]
    wi = [r["warm_iters"] for r in res]
    cs = [r["cold_s"] for r in res]
    ws = [r["warm_s"] for r in res]
    out = {"workload": w.name, "network_params": net.nparam, "train_steps": train_steps,
           "train_s": round(train_s, 2), "train_ms_per_step": round(1e3 * train_s / max(1, train_steps), 3),
           "validation_loss": [[j, v] for j, v in val_loss], "validation_samples": n_val,
           "eval_samples": n_eval,
           "cold_iters_mean": float(np.mean(ci)), "warm_iters_mean": float(np.mean(wi)),
           "iters_ratio": round(float(np.sum(wi) / np.sum(ci)), 4),
           "cold_s_mean": float(np.mean(cs)), "warm_s_mean": float(np.mean(ws)),
           "speedup": round(float(np.sum(cs) / np.sum(ws)), 4),
           "oracle_objective_cold_mean": float(np.mean(obj_c)), "oracle_objective_warm_mean": float(np.mean(obj_w)),
           "oracle_objective_warm_over_cold": [round(a / c, 6) for a, c in zip(obj_w, obj_c)],
           "rel_l2_to_tight_minimiser_cold": [round(v, 5) for v in dist_c],
           "rel_l2_to_tight_minimiser_warm": [round(v, 5) for v in dist_w],
           "tight_minimiser_samples": n_tight, "tight_minimiser_iters": tight_it,
           "tight_minimiser_rel_step": tight_r,
           "truth_rel_l2_cold_warm_init_mean": [
               round(float(np.mean([float((r[k] - r["truth"]).norm() / r["truth"].norm()) for r in res])), 5)
               for k in ("cold", "warm", "init")],
           "note": "both solves stop at the same r_k <= %g (the warm time includes the back-projections and "
                   "the network); the end points are not the same image: the objective and the distance to the "
                   "tight minimiser (the solver continued from the cold end point to r_k <= 1e-7 or %d updates, "
                   "on the first %d samples) say how close each is" % (tol, tight_iters, n_tight)}
    return out


def pmc_driver(args):
    """Counter-run driver: the workload's plan, 20 A+A^T steps as the bench times them
    and 20 as separate forward and adjoint calls, then 5 device copies of 256 MiB (the
    calibration kernel of known size)."""
    import torch
    from paper_2503_13802_amd import inputs, mh3d
    w = inputs.workload(args.workload)
    plan = mh3d.Plan(w.shape, w.harmonics, w.a_per_mm, w.ds, w.sigma_mm, w.lam, w.voxel_mm)
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
    print("pmc driver: %s tiles %s path %d, 20 fused and 20 separate A+A^T steps, 5 copies of 256 MiB"
          % (w.name, plan.tiles(), plan.path()), flush=True)


def net_driver(args):
    """Trace driver for the warm-start network at the workload's shape: 20 training steps
    on 64^3 crops (phantom, portraits, back-projections, loss and gradients, Adam) and 5
    start images (back-projections and the forward pass over the whole volume)."""
    import torch
    from paper_2503_13802_amd import inputs, mh3d
    w = inputs.workload(args.workload)
    plan = mh3d.Plan(w.shape, w.harmonics, w.a_per_mm, w.ds, w.sigma_mm, w.lam, w.voxel_mm)
    net = mh3d.Net(WARM_WIDTHS, in_channels=len(w.harmonics), seed=0)
    rho = plan.phantom(11)
    d = plan.noisy_data(rho, 11, 30.0)
    x = plan.backproject(d)
    crop = [0, 0, 0, 64, 64, 64]
    for _ in range(20):
        net.loss_grad(x, rho, crop, want_loss=False)
        net.adam_step(1e-3)
    for _ in range(5):
        net.warm_start(plan, d)
    torch.cuda.synchronize()
    print("net driver: %s, widths %s, 20 training steps on 64^3 crops, 5 start images"
          % (w.name, list(WARM_WIDTHS)), flush=True)


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


WARM_WIDTHS = (8, 16, 32, 80)   # the warm-start U-Net's channel widths per level (about 0.46 M parameters)

PAPER_CONTEXT = {
    "source": "Table tab:runtime (Sec. 4.3): MATLAB on an NVIDIA GeForce RTX 3070 Laptop GPU, 4 harmonics, "
              "500 iterations of the accelerated projected gradient (one A and one A^T each)",
    "rows": [{"grid": [100, 100, 121], "total_s": 27.0, "A_plus_AT_per_s": 18.5},
             {"grid": [100, 100, 151], "total_s": 35.0, "A_plus_AT_per_s": 14.3},
             {"grid": [100, 100, 241], "total_s": 46.4, "A_plus_AT_per_s": 10.8}],
    "note": "another machine, another grid and harmonic count: context, not a target"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", type=int, default=2, choices=[1, 2])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-volumes", type=int, default=64)
    ap.add_argument("--no-warm", action="store_true")
    ap.add_argument("--no-vector", action="store_true")
    ap.add_argument("--no-mh2d", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="heuristic tiles instead of the autotuner")
    ap.add_argument("--tile-cache", default=None, help="autotuner JSON cache (default: a file in the temp dir)")
    ap.add_argument("--warm-train-steps", type=int, default=20000)
    ap.add_argument("--warm-eval", type=int, default=32)
    ap.add_argument("--pmc-driver", action="store_true",
                    help="only run the workload's A+A^T steps and a copy of known size (for counter runs)")
    ap.add_argument("--net-driver", action="store_true",
                    help="only run warm-start network training steps and start images (for kernel traces)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only; more GPUs would each take whole volumes of a batch "
              "with no exchange between them, which is not implemented", file=sys.stderr)
        sys.exit(2)

    import multiprocessing as mp
    import numpy as np
    from paper_2503_13802_amd import inputs

    if args.pmc_driver:
        pmc_driver(args)
        return
    if args.net_driver:
        net_driver(args)
        return

    # CPU work started before the GPU is touched: the batch's host phantoms (a pool) and
    # the oracle process (data, step sizes and reconstructions of the solve legs)
    batch_inputs = None
    if not args.no_batch:
        bws = inputs.batch_workloads(args.batch_volumes)
        t0 = time.perf_counter()
        with mp.Pool(min(16, os.cpu_count() or 1)) as pool:
            phantoms = pool.map(inputs.phantom, bws)
        batch_inputs = (bws, phantoms, time.perf_counter() - t0)
        log("batch phantoms: %d volumes in %.1f s" % (len(bws), batch_inputs[2]))
    oracle = None
    solve_wls = []
    if not args.no_solve:
        solve_wls.append(args.workload)
        if not args.no_secondary and args.workload != 1:
            solve_wls.append(1)
        q = mp.Queue()
        proc = mp.Process(target=oracle_jobs, args=(solve_wls, q, max(1, (os.cpu_count() or 4) - 4)), daemon=True)
        proc.start()
        oracle = OracleResults(q, proc)
        Quiet.oracle = oracle

    import torch
    w = inputs.workload(args.workload)
    tile_cache = None if args.no_tune else tile_cache_path(args.tile_cache)
    log("workload %s" % w.name)
    plan, op = operator_leg(w, args.steps, args.warmup, tile_cache)
    log("%s: %.1f A+A^T/s fused, %.1f separate; kernels %s" % (w.name, op["rate"], op["separate_rate"],
                                                               json.dumps(op["kernels_us"])))
    out = {
        "metric": "A+A^T applications/s & time-to-recon at rel.residual 1e-4 (plain vs warm/batched)",
        "value": round(op["rate"], 2),
        "unit": "A+A^T applications/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(op["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": list(w.shape), "harmonics": list(w.harmonics),
                   "decimation": list(w.ds), "a_per_mm": w.a_per_mm, "lambda": w.lam,
                   "step": "A then A^T of its own output (d written to HBM), three launches"},
        "roofline": op["roofline"],
        "independent_A_plus_AT_per_s": round(op["separate_rate"], 2),
        "headline_is": "the fused step (A rho, then A^T of that d); independent_A_plus_AT_per_s is A and A^T "
                       "as separate calls on independent inputs",
    }
    for k in ("kernels_us_in_step", "kernels_us", "kernel_bytes_per_launch", "operator_bytes_per_application",
              "operator_GBps", "path", "plan_s", "tiles", "oracle_rel_l2"):
        out[k] = op[k]

    if not args.no_vector:
        w1 = inputs.workload(1)
        out["vector_model"] = vector_leg(w1, min(args.steps, 200), min(args.warmup, 20), tile_cache)
    if not args.no_mh2d:
        out["mh2d"] = mh2d_leg(min(args.steps, 200), min(args.warmup, 20), tile_cache)
    d_main = None
    if not args.no_solve:
        log("plain solve of %s to r <= %g" % (w.name, w.tol))
        out["time_to_recon"], d_main = solve_leg(plan, w, oracle, args.workload)
    if batch_inputs is not None:
        out["batched"] = batched_leg(batch_inputs, 1e-4, 5000, tile_cache)
    if not args.no_warm:
        out["warm_start"] = warm_leg(args.warm_train_steps, args.warm_eval, w.tol, w.max_iter, tile_cache)
    if d_main is not None:
        log("oracle reconstruction of %s" % w.name)
        out["time_to_recon"]["oracle"] = solve_check(plan, w, oracle, args.workload, d_main)
    plan.close()
    if not args.no_secondary and args.workload != 1:
        w1 = inputs.workload(1)
        # the secondary workload: the median of three timed loops (the headline times one)
        p1, op1 = operator_leg(w1, min(args.steps, 200), min(args.warmup, 20), tile_cache, repeats=3)
        sec = {"workload": w1.name, "grid": list(w1.shape), "harmonics": list(w1.harmonics),
               "decimation": list(w1.ds), "A_plus_AT_per_s": round(op1["rate"], 2),
               "independent_A_plus_AT_per_s": round(op1["separate_rate"], 2),
               "timing": "median of 3 loops of the steps"}
        for k in ("roofline", "kernels_us_in_step", "kernels_us", "path", "tiles", "oracle_rel_l2"):
            sec[k] = op1[k]
        if not args.no_solve:
            sec["time_to_recon"], d1 = solve_leg(p1, w1, oracle, 1)
            sec["time_to_recon"]["oracle"] = solve_check(p1, w1, oracle, 1, d1)
        p1.close()
        out["secondary"] = sec
    if oracle is not None:
        oracle.join()
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w, inputs.phantom(w), inputs.noise_draw(w))
    out["paper_context"] = PAPER_CONTEXT
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
