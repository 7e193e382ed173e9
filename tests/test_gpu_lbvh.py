"""The BVH built on the GPU (linear BVH, rr_bvh_options.builder = 1) and its
refit, through the C ABI.

The closest hit is the minimum of (t, original triangle id) over the scene,
whatever the tree, so a scan over the GPU-built tree must give the same path
records as the oracle's brute force, and the same fixed-point accumulator,
bit for bit, as a scan over the host-built SAH tree.  The downloaded tree is
also checked on the host: host traversal against brute force over its
leaves, and every hittable triangle in exactly one leaf.
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


def scan(R, ctx, sc, s, params=None, pose=None, mask=None):
    import torch
    m = None if mask is None else torch.from_numpy(np.ascontiguousarray(mask, dtype=np.uint8)).cuda()
    out = R.rr_radar_scan_records(ctx.handle, sc.handle, pose or s.pose, params or s.params, s.materials,
                                  primary_mask=m)
    torch.cuda.synchronize()
    return dict(image=out["image"].cpu().numpy(), records=out["records"].cpu().numpy(),
                accum=out["accum"].cpu().numpy(), stats=out["stats"])


def deep_mesh():
    n = 5000
    xs = np.minimum(np.cumsum(1.05 ** np.arange(n)) * 1e-3, 1e6)
    V = np.zeros((3 * n, 3), np.float32)
    V[0::3, 0] = xs
    V[1::3, 0] = xs + 1e-3
    V[1::3, 1] = 0.5
    V[2::3, 0] = xs
    V[2::3, 2] = 0.5
    return W.Scene("deep", V, np.arange(3 * n, dtype=np.uint32).reshape(n, 3), np.zeros(n, np.uint16),
                   [W.material_lambertian(0.5)], W.identity_pose(), W.tiny_room().params)


SCENES = {
    "tiny_room": lambda: W.tiny_room(),
    "urban_block": lambda: W.urban_block(),
    "large_scene": lambda: W.large_scene(),
    "thin_pillars": lambda: W.thin_pillars_scene(),
    "single": lambda: W.single_triangle_scene((3, -2, -2), (3, 0, 3), (3, 2, -2), W.material_metal()),
    "deep": deep_mesh,
}


@pytest.mark.parametrize("name", list(SCENES))
def test_gpu_built_tree_selfcheck(R, ctx, name):
    s = SCENES[name]()
    log("case: GPU-built tree", name, s.n_tris, "triangles")
    sc = R.Scene(ctx, s.vertices, s.indices, s.tri_material, builder=1)
    try:
        info = sc.info()
        log(f"  nodes {info['n_nodes']}, leaves {info['n_leaves']}, depth {info['max_depth']}, "
            f"stack bound {info['max_stack']}, build {info['build_ms']:.2f} ms")
        assert info["n_tris"] == s.n_tris and info["max_stack"] <= 96
        assert sc.selfcheck(3000 if s.n_tris > 100000 else 20000, 5) == 0
    finally:
        sc.release()


def test_empty_and_degenerate_only(R, ctx):
    s = W.tiny_room(n_azimuth=16, rays_per_beam=8)
    cases = [(s.vertices, s.indices[:0], s.tri_material[:0]),
             (np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0]], np.float32), np.array([[0, 1, 2]], np.uint32),
              np.zeros(1, np.uint16))]
    for V, F, M in cases:
        sc = R.Scene(ctx, V, F, M, builder=1)
        try:
            assert sc.info()["n_hittable"] == 0 and sc.selfcheck(1000, 3) == 0
            out = scan(R, ctx, sc, W.Scene("x", V, F, M, s.materials[:1], s.pose, s.params))
            assert not out["image"].any() and (out["records"][:, 0] == -1).all()
        finally:
            sc.release()


@pytest.mark.parametrize("leaf", [1, 2, 4, 16])
def test_scan_equals_host_tree_tiny_room(R, ctx, leaf):
    s = W.tiny_room()
    a = R.Scene(ctx, s.vertices, s.indices, s.tri_material)
    b = R.Scene(ctx, s.vertices, s.indices, s.tri_material, builder=1, max_leaf_size=leaf)
    try:
        ra, rb = scan(R, ctx, a, s), scan(R, ctx, b, s)
        assert np.array_equal(ra["records"], rb["records"])
        assert np.array_equal(ra["accum"], rb["accum"])
        ref = oracle.scan_scene(s, records=True, exempt=True, threads=8)
        ok = ~ref["exempt"]
        assert not (rb["records"][ok] != ref["records"][ok]).any()
    finally:
        a.release()
        b.release()


@pytest.mark.parametrize("name", ["urban_block", "large_scene"])
def test_scan_equals_host_tree_full_size(R, ctx, name):
    """The spec workload and the 2 M-triangle scene: same records and
    accumulator over the GPU-built tree as over the host SAH tree."""
    s = SCENES[name]()
    mask = None
    if name == "large_scene":
        rng = np.random.default_rng(7)
        n = s.params["n_azimuth"] * s.params["rays_per_beam"]
        mask = (rng.random(n) < 0.05).astype(np.uint8)
    log("case: full-size scan over both trees", name)
    a = R.Scene(ctx, s.vertices, s.indices, s.tri_material)
    b = R.Scene(ctx, s.vertices, s.indices, s.tri_material, builder=1)
    try:
        ra, rb = scan(R, ctx, a, s, mask=mask), scan(R, ctx, b, s, mask=mask)
        assert np.array_equal(ra["records"], rb["records"])
        assert np.array_equal(ra["accum"], rb["accum"])
        assert ra["stats"]["segments"] == rb["stats"]["segments"]
    finally:
        a.release()
        b.release()


def moved(s, t):
    """Frame t of the tiny room with its cuboids moving: each object (12
    triangles after the room's 12) turns about its own vertical axis and
    slides along x."""
    V = s.vertices.astype(np.float64).copy()
    obj_vertices = np.unique(s.indices[12:].reshape(-1))
    n_obj = (s.n_tris - 12) // 12
    for k in range(n_obj):
        vid = np.unique(s.indices[12 + 12 * k: 24 + 12 * k].reshape(-1))
        c = V[vid].mean(axis=0)
        a = 0.15 * t * (1 + k)
        rot = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
        V[vid] = (V[vid] - c) @ rot.T + c + np.array([0.2 * t * (-1) ** k, 0.0, 0.0])
    assert len(obj_vertices) > 0
    return V.astype(np.float32)


def test_refit_follows_moving_objects(R, ctx):
    import torch
    s = W.tiny_room()
    sc = R.Scene(ctx, s.vertices, s.indices, s.tri_material, builder=1)
    try:
        # a refit of a GPU-built tree allocates no device memory
        V0, V1 = torch.from_numpy(s.vertices).cuda(), torch.from_numpy(moved(s, 1)).cuda()
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for V in (V1, V0):
            sc.refit(V)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        for t in (1, 2, 3):
            Vt = moved(s, t)
            sc.refit(torch.from_numpy(Vt).cuda())
            st = W.Scene("moved", Vt, s.indices, s.tri_material, s.materials, s.pose, s.params)
            got = scan(R, ctx, sc, st)
            fresh = R.Scene(ctx, Vt, s.indices, s.tri_material)
            try:
                want = scan(R, ctx, fresh, st)
            finally:
                fresh.release()
            assert np.array_equal(got["records"], want["records"]), t
            assert np.array_equal(got["accum"], want["accum"]), t
            ref = oracle.scan_scene(st, records=True, exempt=True, threads=8)
            ok = ~ref["exempt"]
            assert not (got["records"][ok] != ref["records"][ok]).any(), t
            assert sc.selfcheck(20000, t) == 0
            log(f"  frame {t}: records equal the oracle on {int(ok.sum())} primaries")
    finally:
        sc.release()


def test_spatial_split_trees_keep_records(R, ctx):
    """Trees without spatial splits, with the default budget and with a large
    one give the urban block the same hit records, accumulator and image
    bit for bit: a triangle referenced by several leaves is hit at the same
    (t, original id) wherever it is tested."""
    s = W.urban_block()
    runs = {}
    for sp in (-1, 0, 100):
        sc = R.Scene(ctx, s.vertices, s.indices, s.tri_material, spatial_pct=sp)
        try:
            info = sc.info()
            runs[sp] = scan(R, ctx, sc, s)
            log(f"  spatial_pct {sp}: {info['n_nodes']} nodes, {info['n_leaves']} leaves, "
                f"cost {info['sah_cost']:.3f}")
        finally:
            sc.release()
    for sp in (0, 100):
        for k in ("records", "accum", "image"):
            assert np.array_equal(runs[sp][k], runs[-1][k]), (sp, k)


@pytest.mark.parametrize("opts", [dict(), dict(collapse=1), dict(merge_leaves=2, max_leaf_size=4),
                                  dict(split_pct=50), dict(spatial_pct=-1)],
                         ids=["optimal", "greedy", "binary-leaves", "split", "no-spatial"])
def test_host_tree_refit_follows_moving_objects(R, ctx, opts):
    """A host-built SAH tree refitted on the GPU: scans over it give the
    records and accumulator of a fresh host build over the moved vertices
    (the closest hit does not depend on the tree) and the oracle's records;
    a refit back to the build's vertices gives the first scan again."""
    import torch
    s = W.tiny_room()
    sc = R.Scene(ctx, s.vertices, s.indices, s.tri_material, **opts)
    try:
        first = scan(R, ctx, sc, s)
        for t in (1, 3):
            Vt = moved(s, t)
            sc.refit(torch.from_numpy(Vt).cuda())
            st = W.Scene("moved", Vt, s.indices, s.tri_material, s.materials, s.pose, s.params)
            got = scan(R, ctx, sc, st)
            fresh = R.Scene(ctx, Vt, s.indices, s.tri_material, **opts)
            try:
                want = scan(R, ctx, fresh, st)
            finally:
                fresh.release()
            assert np.array_equal(got["records"], want["records"]), t
            assert np.array_equal(got["accum"], want["accum"]), t
            ref = oracle.scan_scene(st, records=True, exempt=True, threads=8)
            ok = ~ref["exempt"]
            assert not (got["records"][ok] != ref["records"][ok]).any(), t
            assert sc.selfcheck(20000, t) == 0
            log(f"  {opts} frame {t}: records equal a fresh build and the oracle")
        sc.refit(torch.from_numpy(s.vertices).cuda())
        again = scan(R, ctx, sc, s)
        for k in ("records", "accum", "image"):
            assert np.array_equal(again[k], first[k]), k
    finally:
        sc.release()


def test_host_tree_refit_urban_block(R, ctx):
    """The urban block (about 200k triangles) moved by a small scale and
    shift, refitted on the GPU: the scan equals one over a fresh host build,
    bit for bit.  Refits after the first allocate no device memory."""
    import torch
    s = W.urban_block(n_azimuth=64)
    sc = R.Scene(ctx, s.vertices, s.indices, s.tri_material)
    try:
        Vt = (s.vertices.astype(np.float64) * 1.01 + np.array([0.3, -0.2, 0.05])).astype(np.float32)
        V0, V1 = torch.from_numpy(s.vertices).cuda(), torch.from_numpy(Vt).cuda()
        sc.refit(V0)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for V in (V1, V0, V1):
            sc.refit(V)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        st = W.Scene("moved", Vt, s.indices, s.tri_material, s.materials, s.pose, s.params)
        got = scan(R, ctx, sc, st)
        fresh = R.Scene(ctx, Vt, s.indices, s.tri_material)
        try:
            want = scan(R, ctx, fresh, st)
        finally:
            fresh.release()
        for k in ("records", "accum", "image"):
            assert np.array_equal(got[k], want[k]), k
        assert got["stats"]["segments"] == want["stats"]["segments"]
        assert sc.selfcheck(3000, 5) == 0
    finally:
        sc.release()


@pytest.mark.parametrize("builder", [0, 1])
def test_refit_with_triangles_made_degenerate(R, ctx, builder):
    """A refit that flattens one cuboid onto a plane and collapses an edge of
    another makes some triangles exactly degenerate: they stay in their
    leaves but are never hit, so the scan equals one over a fresh host build
    (which leaves them out) and the oracle's records."""
    import torch
    s = W.tiny_room()
    V = s.vertices.copy()
    a = np.unique(s.indices[12:24].reshape(-1))
    V[a, 0] = V[a, 0].mean(dtype=np.float64).astype(np.float32)
    f = s.indices[24]
    V[f[1]] = V[f[0]]
    sc = R.Scene(ctx, s.vertices, s.indices, s.tri_material, builder=builder)
    try:
        sc.refit(torch.from_numpy(V).cuda())
        st = W.Scene("flattened", V, s.indices, s.tri_material, s.materials, s.pose, s.params)
        got = scan(R, ctx, sc, st)
        fresh = R.Scene(ctx, V, s.indices, s.tri_material)
        try:
            assert fresh.info()["n_hittable"] < s.n_tris
            want = scan(R, ctx, fresh, st)
        finally:
            fresh.release()
        assert np.array_equal(got["records"], want["records"])
        assert np.array_equal(got["accum"], want["accum"])
        ref = oracle.scan_scene(st, records=True, exempt=True, threads=8)
        ok = ~ref["exempt"]
        assert not (got["records"][ok] != ref["records"][ok]).any()
        assert sc.selfcheck(20000, 9) == 0
    finally:
        sc.release()


def test_refit_errors(R, ctx):
    import torch
    s = W.tiny_room(n_azimuth=8, rays_per_beam=4)
    host = R.Scene(ctx, s.vertices, s.indices, s.tri_material)
    wide = R.Scene(ctx, s.vertices, s.indices, s.tri_material, width=8, max_leaf_size=2)
    gpu = R.Scene(ctx, s.vertices, s.indices, s.tri_material, builder=1)
    try:
        V = torch.from_numpy(s.vertices).cuda()
        with pytest.raises(R.RadarError) as e:
            wide.refit(V)
        assert e.value.status == R.RR_EINVAL
        for sc in (host, gpu):
            with pytest.raises(R.RadarError) as e:
                sc.refit(V[:-1].contiguous())
            assert e.value.status == R.RR_EINVAL
    finally:
        host.release()
        wide.release()
        gpu.release()
