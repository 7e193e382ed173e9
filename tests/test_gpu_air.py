"""GPU parity of the air-path (multi-path) returns (Sec. III-A, second return
path) through the C ABI against the oracle on the same seeded scenes.

Bar: as for the retrace path.  Hit records, and the air-path outcome of every
hit (none / returned / blocked / beyond the last bin), are equal for every
primary the oracle does not flag as near-degenerate; the image is within
relative L2 1e-4 of the oracle's float64 image.  Batches and graph replays
equal single scans bit for bit.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from test_oracle_air_pins import GLOSSY, mirror_floor

pytestmark = pytest.mark.gpu

REL_L2 = 1e-4
AIR = W.FLAG_AIR_PATH


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


def gpu_run(R, ctx, scene, params, mask=None):
    import torch
    sc = R.Scene(ctx, scene.vertices, scene.indices, scene.tri_material)
    try:
        m = None
        if mask is not None:
            m = torch.from_numpy(np.ascontiguousarray(mask, dtype=np.uint8)).cuda()
        out = R.rr_radar_scan_records(ctx.handle, sc.handle, scene.pose, params, scene.materials, primary_mask=m)
        torch.cuda.synchronize()
        return dict(image=out["image"].cpu().numpy().astype(np.float64), records=out["records"].cpu().numpy(),
                    air=out["air_records"].cpu().numpy(), accum=out["accum"].cpu().numpy(), stats=out["stats"])
    finally:
        sc.release()


def compare(gpu, ref, cols, n_s, label, mask=None):
    rows = np.concatenate([np.arange(c * n_s, (c + 1) * n_s) for c in cols])
    ok = ~ref["exempt"]
    if mask is not None:
        ok &= mask[rows].astype(bool)
    bad_hit = (gpu["records"][rows] != ref["records"]).any(axis=1) & ok
    bad_air = (gpu["air"][rows] != ref["air_records"]).any(axis=1) & ok
    img = gpu["image"][cols]
    nb = np.linalg.norm(ref["image"])
    rel = float(np.linalg.norm(img - ref["image"]) / nb) if nb > 0 else float(np.linalg.norm(img))
    outcomes = {v: int((ref["air_records"][ok] == v).sum()) for v in (0, 1, 2)}
    log(f"{label}: {int(ok.sum())} primaries, {int(bad_hit.sum())} hit / {int(bad_air.sum())} air records differ, "
        f"{int(ref['exempt'].sum())} exempt, air outcomes {outcomes}, image rel-L2 {rel:.3e}")
    if bad_air.any():
        i = int(np.nonzero(bad_air)[0][0])
        log("  first differing air record", int(rows[i]), gpu["air"][rows][i].tolist(), ref["air_records"][i].tolist())
    assert not bad_hit.any() and not bad_air.any()
    assert rel <= REL_L2
    return outcomes


@pytest.mark.parametrize("case", ["gain", "no_gain", "b5", "return_all", "rotated", "b10"])
def test_air_tiny_room(R, ctx, case):
    kw = dict(n_azimuth=400, rays_per_beam=64, max_bounces=3)
    if case == "b5":
        kw.update(n_azimuth=96, rays_per_beam=16, max_bounces=5)
    if case == "b10":
        kw.update(n_azimuth=96, rays_per_beam=16, beam_width_deg=10.0)
    s = W.tiny_room(**kw)
    flags = {"gain": W.FLAG_BEAM_GAIN, "no_gain": 0, "return_all": W.FLAG_BEAM_GAIN | W.FLAG_RETURN_ALL}.get(
        case, W.FLAG_BEAM_GAIN)
    if case == "rotated":
        s.pose = dict(position=(0.3, -0.2, 0.4), quat_wxyz=tuple(
            np.array([0.95, 0.05, -0.1, 0.28]) / np.linalg.norm([0.95, 0.05, -0.1, 0.28])))
    p = dict(s.params, flags=flags | AIR)
    log("case: tiny room air path", case)
    gpu = gpu_run(R, ctx, s, p)
    ref = oracle.scan_scene(s, params=p, records=True, exempt=True, threads=8)
    out = compare(gpu, ref, list(range(p["n_azimuth"])), p["rays_per_beam"], case)
    # (with every reflected share returned along the retrace path, only
    # refracted children reach depth 1 and nothing is left for the air path)
    assert out[1] > 0 and (out[0] > 0 or case == "return_all")
    assert gpu["stats"]["segments"] == int(ref["segments"].sum())
    assert gpu["stats"]["overflow"] == 0


@pytest.mark.parametrize("floor", ["lambertian", "glossy"])
def test_air_mirror_floor_with_blocker(R, ctx, floor):
    s = mirror_floor(with_blocker=True, gain=True, floor=GLOSSY if floor == "glossy" else None)
    p = dict(s.params, flags=s.params["flags"] | AIR)
    log("case: mirror and floor with a blocker", floor)
    gpu = gpu_run(R, ctx, s, p)
    ref = oracle.scan_scene(s, params=p, records=True, exempt=True)
    out = compare(gpu, ref, [0], p["rays_per_beam"], "mirror/floor " + floor)
    assert out[0] > 100 and out[1] > 10


def test_air_urban_block_columns(R, ctx):
    s = W.urban_block()
    p = dict(s.params, flags=s.params["flags"] | AIR)
    n_s = p["rays_per_beam"]
    log("case: urban block 400 x 1024, B = 4, air path, oracle on 4 columns")
    gpu = gpu_run(R, ctx, s, p)
    cols = [0, 113, 229, 331]
    ref = oracle.scan_scene(s, params=p, columns=cols, records=True, exempt=True)
    out = compare(gpu, ref, cols, n_s, "urban block air")
    assert out[0] > 0 and out[1] > 0
    assert gpu["stats"]["overflow"] == 0


def test_air_bit_reproducible_and_batch_equals_single(R, ctx):
    import torch
    s = W.tiny_room()
    p = dict(s.params, flags=s.params["flags"] | AIR)
    a, b = gpu_run(R, ctx, s, p), gpu_run(R, ctx, s, p)
    assert np.array_equal(a["accum"], b["accum"]) and np.array_equal(a["air"], b["air"])
    scans = []
    for i, (naz, ns, nb, air) in enumerate([(100, 16, 2, True), (400, 64, 3, False), (37, 5, 4, True),
                                            (64, 8, 3, True)]):
        q = dict(s.params, n_azimuth=naz, rays_per_beam=ns, max_bounces=nb, scan_id=i,
                 flags=s.params["flags"] | (AIR if air else 0))
        scans.append((W.yaw_pose((0.2 * i, -0.1 * i, 0.0), 0.3 * i), q))
    sc = R.Scene(ctx, s.vertices, s.indices, s.tri_material)
    try:
        imgs, st = R.rr_radar_scan_batch(ctx.handle, sc.handle, scans, s.materials, stats=True)
        for (pose, q), im in zip(scans, imgs):
            one, _ = R.rr_radar_scan(ctx.handle, sc.handle, pose, q, s.materials)
            torch.cuda.synchronize()
            assert torch.equal(one, im)
        assert st["overflow"] == 0
        # a captured graph of the batch replays to the same images
        g, first = R.rr_graph_create(ctx.handle, sc.handle, scans, s.materials)
        try:
            for _ in range(3):
                for x in first:
                    x.fill_(-1.0)
                R.rr_graph_launch(g)
                torch.cuda.synchronize()
                for x, im in zip(first, imgs):
                    assert torch.equal(x, im)
        finally:
            R.rr_graph_destroy(g)
    finally:
        sc.release()


def test_air_needs_four_wide_levels(R, ctx):
    s = W.tiny_room(n_azimuth=8, rays_per_beam=4)
    p = dict(s.params, flags=s.params["flags"] | AIR)
    sc = R.Scene(ctx, s.vertices, s.indices, s.tri_material, width=8)
    try:
        with pytest.raises(R.RadarError) as e:
            R.rr_radar_scan(ctx.handle, sc.handle, s.pose, p, s.materials)
        assert e.value.status == R.RR_EINVAL
    finally:
        sc.release()
    before = R.rr_get_tuning(ctx.handle)
    sc = R.Scene(ctx, s.vertices, s.indices, s.tri_material)
    try:
        R.rr_set_tuning(ctx.handle, fused=1)
        with pytest.raises(R.RadarError) as e:
            R.rr_radar_scan(ctx.handle, sc.handle, s.pose, p, s.materials)
        assert e.value.status == R.RR_EINVAL
    finally:
        R.rr_set_tuning(ctx.handle, **before)
        sc.release()
