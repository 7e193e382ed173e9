"""GPU parity of the polar-image epilogue (Sec. III-B "Polar Image",
Sec. III-C "Noise") through the C ABI against the CPU oracle on the same
seeded images.

Bar: the 8-bit pixels are bit-exact except where the oracle's unrounded pixel
value lies within 1e-9 of a rounding boundary (both sides decide in float64;
only log10 may round differently, by an ulp); the float32 dB values agree to
one float32 ulp, and -inf (zero energy) exactly.  The fused scan + epilogue
equals the scan followed by the stand-alone epilogue bit for bit.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


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


def gpu_post(R, ctx, imgs, post):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(imgs)).cuda()
    db, u8 = R.rr_postprocess(ctx.handle, t, post)
    torch.cuda.synchronize()
    return db.cpu().numpy(), u8.cpu().numpy()


def oracle_post(imgs, post):
    """Per image i, scan id + i, as the batched entry point defines."""
    dbs, u8s, pres = [], [], []
    for i, im in enumerate(imgs):
        p = dict(post, scan_id=(post.get("scan_id", 0) + i) & 0xFFFFFFFF)
        d, u, q = oracle.postprocess(im, p)
        dbs.append(d)
        u8s.append(u)
        pres.append(q)
    return np.stack(dbs), np.stack(u8s), np.stack(pres)


def assert_post_equal(db_g, u8_g, db_o, u8_o, pre_o, what=""):
    # pixels whose pre-rounding value sits on a half (either rounding is
    # correct); pre is -inf where the energy is zero, which is never a tie
    with np.errstate(invalid="ignore"):
        boundary = np.abs(pre_o - (np.floor(pre_o) + 0.5)) < 1e-9
    bad = (u8_g != u8_o) & ~boundary
    assert not bad.any(), f"{what}: {int(bad.sum())} pixels differ, first at {np.argwhere(bad)[0]}"
    assert boundary.mean() < 1e-3
    fin = np.isfinite(db_o)
    assert np.array_equal(np.isfinite(db_g), fin), what
    assert np.array_equal(db_g[~fin], db_o[~fin]), what
    diff = np.abs(db_g[fin].astype(np.float64) - db_o[fin].astype(np.float64))
    ulp = np.spacing(np.abs(db_o[fin])).astype(np.float64)
    assert (diff <= ulp).all(), f"{what}: dB differs by up to {(diff / np.maximum(ulp, 1e-45)).max()} ulp"
    return int(boundary.sum())


POSTS = {
    "plain": dict(),
    "blur_half": dict(blur_sigma_bins=0.5),
    "blur_2": dict(blur_sigma_bins=2.0),
    "blur_max": dict(blur_sigma_bins=16.0),
    "uniform": dict(uniform_amp=1e-6, seed=99),
    "perlin": dict(perlin_amp=1e-5, perlin_cell_az=4.0, perlin_cell_bins=16.0, seed=7),
    "perlin_unit_cells": dict(perlin_amp=1e-5, perlin_cell_az=1.0, perlin_cell_bins=1.0),
    "perlin_odd_cells": dict(perlin_amp=1e-5, perlin_cell_az=2.5, perlin_cell_bins=37.25, scan_id=2**32 - 2),
    "full": dict(blur_sigma_bins=2.0, uniform_amp=1e-7, perlin_amp=1e-6, perlin_cell_az=16.0,
                 perlin_cell_bins=64.0, seed=12345, scan_id=3),
    "floor60": dict(db_floor=-60.0, max_value=200, blur_sigma_bins=1.3, uniform_amp=1e-8),
}
SHAPES = [(1, 1, 1), (1, 3, 1023), (2, 5, 1025), (3, 2, 3776), (1, 7, 4099), (2, 4, 17)]


@pytest.mark.parametrize("name", list(POSTS))
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_postprocess_matches_oracle(R, ctx, name, shape):
    log("postprocess", name, shape)
    imgs = W.polar_images(sum(shape) + len(name), *shape)
    db_g, u8_g = gpu_post(R, ctx, imgs, POSTS[name])
    db_o, u8_o, pre_o = oracle_post(imgs, POSTS[name])
    assert_post_equal(db_g, u8_g, db_o, u8_o, pre_o, f"{name} {shape}")


def test_postprocess_full_size(R, ctx):
    """Two urban-block images (400 x 3776) with every noise on, whole images."""
    post = POSTS["full"]
    imgs = W.polar_images(21, 2, 400, 3776)
    log("postprocess full size")
    db_g, u8_g = gpu_post(R, ctx, imgs, post)
    db_o, u8_o, pre_o = oracle_post(imgs, post)
    n = assert_post_equal(db_g, u8_g, db_o, u8_o, pre_o, "full size")
    log("boundary pixels", n, "of", u8_o.size)


def test_postprocess_outputs_optional_and_batch_offsets(R, ctx):
    import torch
    imgs = torch.from_numpy(W.polar_images(5, 3, 6, 2000)).cuda()
    post = POSTS["full"]
    db, u8 = R.rr_postprocess(ctx.handle, imgs, post)
    db1, none = R.rr_postprocess(ctx.handle, imgs, post, want_u8=False)
    none2, u81 = R.rr_postprocess(ctx.handle, imgs, post, want_db=False)
    assert none is None and none2 is None
    assert torch.equal(db, db1) and torch.equal(u8, u81)
    # image i of a batch is image 0 of a call with scan id + i
    for i in range(3):
        d, u = R.rr_postprocess(ctx.handle, imgs[i].contiguous(), dict(post, scan_id=post["scan_id"] + i))
        assert torch.equal(d, db[i]) and torch.equal(u, u8[i])
    # the same call twice gives the same bytes; another seed other noise
    db2, u82 = R.rr_postprocess(ctx.handle, imgs, post)
    assert torch.equal(db, db2) and torch.equal(u8, u82)
    db3, _ = R.rr_postprocess(ctx.handle, imgs, dict(post, seed=post["seed"] + 1))
    assert not torch.equal(db, db3)


def test_postprocess_empty_and_errors(R, ctx):
    import torch
    e = torch.empty((0, 5, 7), dtype=torch.float32, device="cuda")
    db, u8 = R.rr_postprocess(ctx.handle, e, {})
    assert db.numel() == 0 and u8.numel() == 0
    imgs = torch.zeros((2, 3), dtype=torch.float32, device="cuda")
    lib = R.load_library()
    pp = R.make_post({})
    # an output that overlaps the input
    st = lib.rr_postprocess(ctx.handle, R._ptr(imgs), 1, 2, 3, R.C.byref(pp), R._ptr(imgs), None, None)
    assert st == R.RR_EINVAL
    for bad in (dict(blur_sigma_bins=16.5), dict(db_floor=0.0), dict(max_value=256),
                dict(perlin_amp=1.0, perlin_cell_bins=0.5), dict(uniform_amp=-1.0)):
        with pytest.raises(R.RadarError) as ex:
            R.rr_postprocess(ctx.handle, imgs, bad)
        assert ex.value.status == R.RR_EINVAL


@pytest.mark.parametrize("scene_name", ["tiny_room", "urban_block"])
def test_fused_scan_post_equals_scan_then_post(R, ctx, scene_name):
    import torch
    s = W.tiny_room() if scene_name == "tiny_room" else W.urban_block(rays_per_beam=64)
    post = POSTS["full"]
    sc = R.Scene(ctx, s.vertices, s.indices, s.tri_material)
    try:
        log("fused scan + epilogue", scene_name)
        img, _ = R.rr_radar_scan(ctx.handle, sc.handle, s.pose, s.params, s.materials)
        db, u8 = R.rr_postprocess(ctx.handle, img, post)
        img2, db2, u82, st = R.rr_radar_scan_post(ctx.handle, sc.handle, s.pose, s.params, s.materials,
                                                  post, stats=True)
        torch.cuda.synchronize()
        assert st["overflow"] == 0
        assert torch.equal(img, img2) and torch.equal(db, db2) and torch.equal(u8, u82)
        _, db3, u83, _ = R.rr_radar_scan_post(ctx.handle, sc.handle, s.pose, s.params, s.materials, post,
                                              want_image=False)
        assert torch.equal(db, db3) and torch.equal(u8, u83)
    finally:
        sc.release()


def test_fused_scan_post_against_oracle(R, ctx):
    """Tiny room: the oracle's float64 scan, rounded to float32, through the
    oracle's epilogue, against the fused GPU scan + epilogue.  The two scans
    agree to rounding (fixed-point against float64 sums), so pixels may
    differ by one step where a value sits near a rounding boundary."""
    import torch
    s = W.tiny_room()
    post = dict(blur_sigma_bins=1.5, uniform_amp=1e-9, perlin_amp=1e-8, perlin_cell_az=8.0,
                perlin_cell_bins=32.0, seed=4, scan_id=1)
    ref = oracle.scan_scene(s, energy=False, threads=8)["image"].astype(np.float32)
    db_o, u8_o, pre_o = oracle.postprocess(ref, post)
    sc = R.Scene(ctx, s.vertices, s.indices, s.tri_material)
    try:
        img, db, u8, _ = R.rr_radar_scan_post(ctx.handle, sc.handle, s.pose, s.params, s.materials, post)
        torch.cuda.synchronize()
        img, db, u8 = img.cpu().numpy(), db.cpu().numpy(), u8.cpu().numpy()
    finally:
        sc.release()
    rel = np.linalg.norm(img.astype(np.float64) - ref) / np.linalg.norm(ref)
    assert rel < 1e-4
    d = np.abs(u8.astype(int) - u8_o.astype(int))
    assert d.max() <= 1 and (d > 0).mean() < 1e-3
    fin = np.isfinite(db_o)
    assert np.array_equal(np.isfinite(db), fin)
    assert np.allclose(db[fin], db_o[fin], rtol=0, atol=1e-3)
