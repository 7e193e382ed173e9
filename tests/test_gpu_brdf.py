"""GPU parity of the Cook-Torrance material kind (the user-defined BRDF of
the experiments, Sec. IV) and of the elliptic beam (Sec. III-A) through the
C ABI against the oracle.  Bar: path records equal for every non-exempt
primary, image within relative L2 1e-4."""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

# the parameter set of the paper's Cook-Torrance runs
CT_PAPER = W.material_cook_torrance(0.2, 0.5, 100.0, 0.1)
CT_GLASSY = W.material_cook_torrance(0.05, 0.2, 1.8, 0.5)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2310_03505_amd as lib
    lib.load_library()
    return lib


@pytest.fixture(scope="module")
def ctx(R):
    c = R.Context(0)
    yield c
    c.close()


def run_both(R, ctx, s, params=None, mats=None):
    import torch
    params = params or s.params
    mats = mats or s.materials
    sc = R.Scene(ctx, s.vertices, s.indices, s.tri_material)
    try:
        out = R.rr_radar_scan_records(ctx.handle, sc.handle, s.pose, params, mats)
        torch.cuda.synchronize()
        gpu = dict(image=out["image"].cpu().numpy().astype(np.float64), records=out["records"].cpu().numpy(),
                   accum=out["accum"].cpu().numpy())
        if "air_records" in out:
            gpu["air"] = out["air_records"].cpu().numpy()
    finally:
        sc.release()
    ref = oracle.scan(s.vertices, s.indices, s.tri_material, s.pose, params, mats, records=True, exempt=True,
                      threads=8)
    return gpu, ref


def check(gpu, ref, label):
    ok = ~ref["exempt"]
    bad = (gpu["records"] != ref["records"]).any(axis=1) & ok
    if "air" in gpu:
        bad |= (gpu["air"] != ref["air_records"]).any(axis=1) & ok
    nb = np.linalg.norm(ref["image"])
    rel = float(np.linalg.norm(gpu["image"] - ref["image"]) / nb)
    log(f"{label}: {int(ok.sum())} primaries, {int(bad.sum())} differ, image rel-L2 {rel:.3e}")
    assert not bad.any()
    assert rel <= 1e-4


@pytest.mark.parametrize("case", ["paper_params", "glassy", "with_air_path", "room_walls"])
def test_cook_torrance_tiny_room(R, ctx, case):
    s = W.tiny_room()
    mats = list(s.materials)
    params = s.params
    # materials: 0 walls (Lambertian), 1 metal cuboids, 2 dielectric cuboids
    if case == "paper_params":
        mats[1] = CT_PAPER
    elif case == "glassy":
        mats[2] = CT_GLASSY
    elif case == "with_air_path":
        mats[1] = CT_PAPER
        mats[2] = CT_GLASSY
        params = dict(params, flags=params["flags"] | W.FLAG_AIR_PATH)
    else:
        mats[0] = CT_PAPER
    log("case: Cook-Torrance", case)
    gpu, ref = run_both(R, ctx, s, params, mats)
    check(gpu, ref, case)


def test_cook_torrance_slab_transmits(R, ctx):
    s = W.slab_scene(2.0, 0.05, CT_GLASSY, n_azimuth=4, rays_per_beam=256, max_bounces=3, n_bins=256,
                     bin_size_m=0.044)
    gpu, ref = run_both(R, ctx, s)
    check(gpu, ref, "Cook-Torrance slab")
    assert (ref["records"][:, 2] >= 0).any()


@pytest.mark.parametrize("stretch", [(3.0, 0.5), (0.25, 2.0), (1.0, 1.0)])
def test_elliptic_beam(R, ctx, stretch):
    s = W.tiny_room(beam_width_deg=6.0)
    p = dict(s.params, beam_stretch_az=stretch[0], beam_stretch_inc=stretch[1])
    log("case: elliptic beam", stretch)
    gpu, ref = run_both(R, ctx, s, p)
    check(gpu, ref, f"stretch {stretch}")
    if stretch == (1.0, 1.0):
        plain, _ = run_both(R, ctx, s)
        assert np.array_equal(plain["accum"], gpu["accum"])


def test_validation(R, ctx):
    s = W.tiny_room(n_azimuth=8, rays_per_beam=4)
    sc = R.Scene(ctx, s.vertices, s.indices, s.tri_material)
    try:
        for mats, p in (([dict(CT_PAPER, B=0.0)] + s.materials[1:], s.params),
                        (s.materials, dict(s.params, beam_stretch_az=101.0)),
                        (s.materials, dict(s.params, beam_stretch_inc=-1.0)),
                        ([dict(CT_PAPER, kind=4)] + s.materials[1:], s.params)):
            with pytest.raises(R.RadarError) as e:
                R.rr_radar_scan(ctx.handle, sc.handle, s.pose, p, mats)
            assert e.value.status == R.RR_EINVAL
    finally:
        sc.release()
