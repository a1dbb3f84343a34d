"""Tile shapes of the spectral passes and the autotuner: every valid shape gives the
oracle's operator (the shapes only change the launch decomposition), the tuner's
choice is stored in and read back from its JSON cache, and a batch of tuned plans
still reproduces the single-plan solves exactly."""
import json

import numpy as np
import pytest

from oracle import model as om
from paper_2503_13802_amd import inputs
from gpu_util import announce, rel_l2, torch_cuda

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _valid_E(S):
    out = []
    for e in (1, 2, 3, 4, 6, 8, 9):
        if S % e == 0:
            lg = S // e
            if lg <= 64 and lg & (lg - 1) == 0:
                out.append(e)
    return out


@pytest.mark.parametrize("shape,harm,ds,a,sig", [
    ((12, 8, 16), (2, 3, 5), (2, 2, 4), 0.9, 4.0),
    ((18, 12, 8), (2, 3, 4), (3, 2, 2), 1.0, 5.0),
    ((48, 24, 32), tuple(range(2, 13)), (2, 4, 4), 1.2, 10.0),
])
def test_every_tile_shape_matches_oracle(shape, harm, ds, a, sig):
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    announce("tiles %s ds=%s" % (shape, ds))
    h = om.psf_bank(shape, list(harm), a)
    b = om.sensitivity(shape, sig)
    rho = inputs.random_field(shape, 31)
    d_ref = om.forward_fft(h, b, rho, ds)
    r = inputs.random_field(d_ref.shape, 32)
    x_ref = om.adjoint_fft(h, b, r, ds)
    p = mh3d.Plan(shape, harm, a, ds, sig, 1e-3)
    S = ds[0] * ds[1] * ds[2]
    mx, my, mz = (n // s for n, s in zip(shape, ds))
    ncls = my * (mz // 2 + 1)
    tried = 0
    for E in _valid_E(S):
        for cpw in [c for c in range(1, ncls + 1) if ncls % c == 0][:4]:
            for xb in [x for x in (1, 2, 4) if mx % x == 0]:
                if cpw * mx * S // E > 1024:
                    continue
                ps = (1, 2, 4)[tried % 3]
                try:
                    p.set_tiles(E, cpw, xb, ps)
                except mh3d.MH3DError as e:       # shape exceeds the LDS budget
                    assert "LDS" in str(e)
                    continue
                assert p.tiles() == (E, cpw, xb, ps)
                d = p.forward(torch.tensor(rho, dtype=torch.float32)).cpu().numpy()
                x = p.adjoint(torch.tensor(r, dtype=torch.float32)).cpu().numpy()
                assert rel_l2(d, d_ref) <= TOL, (E, cpw, xb)
                assert rel_l2(x, x_ref) <= TOL, (E, cpw, xb)
                tried += 1
    assert tried >= 4
    from paper_2503_13802_amd.mh3d import MH3DError
    with pytest.raises(MH3DError):
        p.set_tiles(E=5 if S % 5 else 7)       # not a valid split of S
    with pytest.raises(MH3DError):
        p.set_tiles(ps=5)


def test_autotune_cache_round_trip(tmp_path):
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    announce("autotune cache")
    w = inputs.workload(1)
    cache = tmp_path / "tiles.json"
    p = mh3d.Plan(w.shape, w.harmonics, w.a_per_mm, w.ds, w.sigma_mm, w.lam)
    default = p.tiles()
    tiles, us = p.autotune(str(cache))
    assert us > 0 and p.tiles() == tiles
    stored = json.loads(cache.read_text())
    # the plan runs the compile-time passes, but a batch would run the general ones: the
    # general tiles are tuned (and stored) first, then xb on the compile-time passes
    assert sorted(k.split("|", 1)[1] for k in stored) == ["96x96x64|K7|ds2x2x2|analytic",
                                                          "96x96x64|K7|ds2x2x2|analytic|compiled"]
    ent = next(v for k, v in stored.items() if k.endswith("|compiled"))
    gen = next(v for k, v in stored.items() if not k.endswith("|compiled"))
    assert (ent["E"], ent["cpw"], ent["xb"], ent["ps"]) == tiles and ent["xb"] in (1, 2, 4, 8)
    assert all(ent[f] == gen[f] for f in ("E", "cpw", "ps", "ps_solve", "tm"))
    assert ent["ps_solve"] in (1, 2, 4) and ent["tm"] in (512, 1024)
    assert p.path() == 1
    # a second plan of the same geometry reads the cache without timing
    q = mh3d.Plan(w.shape, w.harmonics, w.a_per_mm, w.ds, w.sigma_mm, w.lam)
    tiles2, us2 = q.autotune(str(cache))
    assert tiles2 == tiles and us2 == pytest.approx(ent["us"], abs=1e-3)
    # the tuned plan still matches the default-tile plan on A and A^T
    x = torch.tensor(inputs.random_field(w.shape, 4), dtype=torch.float32, device="cuda")
    p.set_tiles(*default)
    d0 = p.forward(x).cpu().numpy()
    d1 = q.forward(x).cpu().numpy()
    assert rel_l2(d1, d0) <= 2e-6


def test_batch_of_tuned_plans_reproduces_single_solves(tmp_path):
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    announce("batch of tuned plans")
    specs = [((32, 32, 32), (2, 3)), ((48, 24, 32), (2, 3, 4, 5)), ((32, 32, 32), (2, 3))]
    plans, ds = [], []
    for i, (shape, harm) in enumerate(specs):
        p = mh3d.Plan(shape, harm, 0.9, (2, 2, 2), 10.0, 1e-3)
        p.autotune(str(tmp_path / "t.json"))
        rho = torch.tensor(inputs.random_field(shape, 40 + i), dtype=torch.float32, device="cuda").abs()
        ds.append(p.forward(rho))
        plans.append(p)
    single = [p.solve(d, max_iter=60, tol=1e-4, tau=0.0) for p, d in zip(plans, ds)]
    batch = mh3d.Batch(plans)
    rhos, infos = batch.solve(ds, max_iter=60, tol=1e-4, tau=0.0)
    for (r1, i1), r2, i2 in zip(single, rhos, infos):
        assert i1["iters"] == i2["iters"]
        assert torch.equal(r1, r2)
    from paper_2503_13802_amd.mh3d import MH3DError
    with pytest.raises(MH3DError):
        plans[0].set_tiles()                  # frozen while the batch holds the plan


def test_solver_plane_split_does_not_change_results(tmp_path):
    """The solver's passes (and the forward plane pass of A then A^T) may split x-planes
    over a different number of workgroups than the operator calls (the cache's
    ps_solve).  With a fixed step and count the updates, the normal operator, A then A^T
    and the power iteration's estimate do not depend on it (the FP64 sums only change
    their block partition)."""
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    announce("solver plane split")
    shape, harm, ds = (32, 24, 16), (2, 3, 4), (2, 2, 2)
    cache = tmp_path / "tiles.json"
    p0 = mh3d.Plan(shape, harm, 1.0, ds, 6.0, 1e-3)
    p0.autotune(str(cache))
    (key, ent), = json.loads(cache.read_text()).items()
    rho = torch.tensor(inputs.random_field(shape, 21), dtype=torch.float32, device="cuda").abs()
    d = p0.forward(rho)
    x = torch.tensor(inputs.random_field(shape, 22), dtype=torch.float32, device="cuda")
    outs = []
    for pss in (1, 2, 4):
        # the last plan also runs the merged adjoint launch at the other thread count
        tm = {512: 1024, 1024: 512}[ent["tm"]] if pss == 4 else ent["tm"]
        cache.write_text('{\n  "%s": {"E": %d, "cpw": %d, "xb": %d, "ps": %d, "ps_solve": %d, "tm": %d, "us": %.3f}\n}\n'
                         % (key, ent["E"], ent["cpw"], ent["xb"], ent["ps"], pss, tm, ent["us"]))
        p = mh3d.Plan(shape, harm, 1.0, ds, 6.0, 1e-3)
        p.autotune(str(cache))
        rec, info = p.solve(d, max_iter=25, tol=0.0, tau=0.05)
        assert info["iters"] == 25
        outs.append((rec, p.normal(x), p.power_iteration(30, 1), p.forward_adjoint(x)))
        p.close()
    for rec, nx_, lmax, fa in outs[1:]:
        assert torch.equal(rec, outs[0][0])
        assert torch.equal(nx_, outs[0][1])
        assert lmax == pytest.approx(outs[0][2], rel=1e-12)
        assert torch.equal(fa[0], outs[0][3][0]) and torch.equal(fa[1], outs[0][3][1])


def test_cache_entries_of_earlier_formats_are_read(tmp_path):
    """Cache lines without ps_solve / tm (earlier formats) still apply their tiles without
    timing; the missing fields take their defaults."""
    torch = torch_cuda()
    from paper_2503_13802_amd import mh3d
    announce("tile cache formats")
    shape, harm, ds = (32, 24, 16), (2, 3), (2, 2, 2)
    cache = tmp_path / "tiles.json"
    p0 = mh3d.Plan(shape, harm, 1.0, ds, 6.0, 1e-3)
    p0.autotune(str(cache))
    (key, ent), = json.loads(cache.read_text()).items()
    x = torch.tensor(inputs.random_field(shape, 5), dtype=torch.float32, device="cuda")
    want = p0.forward_adjoint(x)
    lines = ['"%s": {"E": %d, "cpw": %d, "xb": %d, "ps": %d, "us": 12.345}' % (key, ent["E"], ent["cpw"], ent["xb"], ent["ps"]),
             '"%s": {"E": %d, "cpw": %d, "xb": %d, "ps": %d, "ps_solve": %d, "us": 12.345}'
             % (key, ent["E"], ent["cpw"], ent["xb"], ent["ps"], ent["ps_solve"])]
    for line in lines:
        cache.write_text("{\n  " + line + "\n}\n")
        p = mh3d.Plan(shape, harm, 1.0, ds, 6.0, 1e-3)
        tiles, us = p.autotune(str(cache))
        assert tiles == (ent["E"], ent["cpw"], ent["xb"], ent["ps"]) and us == pytest.approx(12.345)
        got = p.forward_adjoint(x)
        assert torch.equal(got[0], want[0]) and torch.equal(got[1], want[1])
        p.close()
