"""Host-side checks of the HIP library that need no GPU: the shared library
loads and exports every symbol its header declares, arguments are
validated, and the host-built BVH agrees with brute force."""
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def R():
    import paper_2310_03505_amd as lib
    lib.load_library()
    return lib


def header_functions():
    txt = open(os.path.join(ROOT, "include", "radarays_hip.h")).read()
    return sorted(set(re.findall(r"^\s*(?:rr_status|const char\*)\s+(rr_\w+)\s*\(", txt, re.M)))


def test_exports_every_declared_symbol(R):
    lib = R.load_library()
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(R.EXPORTS)


def test_status_strings(R):
    lib = R.load_library()
    for s in (0, -1, -2, -3, -4, -5):
        assert lib.rr_status_str(s)


def test_no_device_is_reported(R):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(R.RadarError) as e:
        R.rr_create(0)
    assert e.value.status == R.RR_EDEVICE


def test_workspace_query_and_validation(R):
    p = W.urban_block().params
    n = R.rr_workspace_query(p)
    # two queues of N_p * 2^(B-1) rays of 52 bytes, one 8-byte hit per ray
    # of a level, the accumulator, and the traversal-stack spill area
    # (80 entries x 256 CUs x 32 waves x 64 lanes)
    cap = 400 * 1024 * 8
    want = 2 * cap * 52 + cap * 8 + 400 * 3776 * 8 + 4 * 80 * 256 * 32 * 64
    assert want <= n < want + (1 << 20)
    for bad in [dict(p, max_bounces=9), dict(p, n_azimuth=0), dict(p, beam_prob=0.0),
                dict(p, beam_width_rad=4.0), dict(p, rays_per_beam=(1 << 20) + 1),
                dict(p, n_azimuth=65535, rays_per_beam=4096)]:
        with pytest.raises(R.RadarError) as e:
            R.rr_workspace_query(bad)
        assert e.value.status == R.RR_EINVAL


def test_scene_upload_validation(R):
    V = np.zeros((3, 3), np.float32)
    with pytest.raises(R.RadarError):
        R.rr_scene_upload(None, V, np.array([[0, 1, 3]], np.uint32), np.zeros(1, np.uint16))
    Vn = V.copy()
    Vn[1, 1] = np.nan
    with pytest.raises(R.RadarError):
        R.rr_scene_upload(None, Vn, np.array([[0, 1, 2]], np.uint32), np.zeros(1, np.uint16))


@pytest.mark.parametrize("name", ["tiny_room", "urban_block", "thin_pillars", "slab", "empty",
                                  "single", "degenerate_only"])
def test_host_bvh_matches_brute_force(R, name):
    if name == "tiny_room":
        s, n = W.tiny_room(), 20000
    elif name == "urban_block":
        s, n = W.urban_block(), 1500
    elif name == "thin_pillars":
        s, n = W.thin_pillars_scene(), 20000
    elif name == "slab":
        s, n = W.slab_scene(2.0, 0.01, W.material_dielectric(2.0)), 5000
    elif name == "empty":
        s, n = W.tiny_room(), 100
        s.indices, s.tri_material = s.indices[:0], s.tri_material[:0]
    elif name == "single":
        s, n = W.single_triangle_scene((3, -2, -2), (3, 0, 3), (3, 2, -2), W.material_metal()), 1000
    else:
        V = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0]], np.float32)
        s = W.Scene("deg", V, np.array([[0, 1, 2]], np.uint32), np.zeros(1, np.uint16), [], {}, {})
        n = 100
    sc = R.Scene(None, s.vertices, s.indices, s.tri_material)
    info = sc.info()
    assert info["max_stack"] <= 96
    assert info["n_tris"] == s.n_tris
    if name == "degenerate_only":
        assert info["n_hittable"] == 0
    assert sc.selfcheck(n, 7) == 0
    sc.release()


@pytest.mark.parametrize("leaf,bins", [(1, 4), (2, 8), (8, 32), (16, 64)])
def test_host_bvh_options(R, leaf, bins):
    s = W.tiny_room()
    sc = R.Scene(None, s.vertices, s.indices, s.tri_material, max_leaf_size=leaf, sah_bins=bins)
    assert sc.selfcheck(5000, 3) == 0
    sc.release()


@pytest.mark.parametrize("width,leaf,split,merge", [(8, 4, 0, 0), (8, 2, 0, 0), (8, 1, 0, 0), (4, 4, 50, 2),
                                                    (8, 3, 100, 0), (4, 2, 0, 1), (4, 4, 0, 2)])
def test_host_bvh_wide_and_split(R, width, leaf, split, merge):
    """Eight-wide trees (octant-ordered groups, merged leaves) and early split
    clipping (a triangle in several leaves) find the brute-force closest hit."""
    for s, n in ((W.tiny_room(), 4000), (W.urban_block(), 1000)):
        sc = R.Scene(None, s.vertices, s.indices, s.tri_material, width=width, max_leaf_size=leaf,
                     split_pct=split, merge_leaves=merge)
        info = sc.info()
        assert info["n_tris"] == s.n_tris and info["n_nodes"] > 0
        assert sc.selfcheck(n, 13) == 0
        sc.release()


@pytest.mark.parametrize("collapse,leaf,split,merge", [(1, 2, 0, 1), (2, 2, 0, 1), (2, 1, 0, 1), (2, 4, 0, 1),
                                                       (2, 2, 50, 1), (2, 4, 0, 2), (1, 4, 0, 2)])
def test_host_bvh_collapse(R, collapse, leaf, split, merge):
    """Greedy (1) and cost-optimal (2) four-wide collapses, with leaves formed
    by the collapse or by the binary build, with and without split
    references, find the brute-force closest hit; the default is the
    cost-optimal tree."""
    for s, n in ((W.tiny_room(), 4000), (W.thin_pillars_scene(), 4000), (W.urban_block(), 1000)):
        sc = R.Scene(None, s.vertices, s.indices, s.tri_material, max_leaf_size=leaf, split_pct=split,
                     merge_leaves=merge, collapse=collapse)
        info = sc.info()
        assert info["n_tris"] == s.n_tris and info["n_nodes"] > 0 and info["max_stack"] <= 96
        assert sc.selfcheck(n, 17) == 0
        sc.release()
    s = W.urban_block()
    infos = []
    for c in (0, 2):
        sc = R.Scene(None, s.vertices, s.indices, s.tri_material, max_leaf_size=leaf, split_pct=split,
                     merge_leaves=merge, collapse=c)
        infos.append(sc.info())
        sc.release()
    assert infos[0]["n_nodes"] == infos[1]["n_nodes"] and infos[0]["sah_cost"] == infos[1]["sah_cost"]


def _long_over_clutter(seed=5):
    """Small random triangles in a 20 m box crossed by long diagonal slivers:
    the case spatial splits are for."""
    rng = np.random.default_rng(seed)
    n_small, n_long = 3000, 24
    c = rng.uniform(0.0, 20.0, (n_small, 1, 3))
    small = (c + rng.normal(0.0, 0.15, (n_small, 3, 3))).reshape(-1, 3)
    a = rng.uniform(0.0, 20.0, (n_long, 3))
    b = rng.uniform(0.0, 20.0, (n_long, 3))
    off = rng.normal(0.0, 0.3, (n_long, 3))
    long_ = np.stack([a, b, a + off], axis=1).reshape(-1, 3)
    V = np.concatenate([small, long_]).astype(np.float32)
    n = n_small + n_long
    F = np.arange(3 * n, dtype=np.uint32).reshape(n, 3)
    return V, F, np.zeros(n, np.uint16)


@pytest.mark.parametrize("width,merge", [(4, 0), (4, 2), (8, 0)])
def test_host_bvh_spatial_splits(R, width, merge):
    """Spatial splits (a triangle cut at a plane is referenced by leaves on
    both sides, each bounded by its part) at several budgets find the
    brute-force closest hit; with a budget they lower the tree's
    surface-area cost and add triangle references where large triangles cross
    small ones, and none are added with -1."""
    V, F, M = _long_over_clutter()
    scenes = [(V, F, M, 6000)]
    for s, n in ((W.tiny_room(), 3000), (W.thin_pillars_scene(), 3000), (W.urban_block(), 800)):
        scenes.append((s.vertices, s.indices, s.tri_material, n))
    for k, (v, f, m, n) in enumerate(scenes):
        infos = {}
        for sp in (-1, 10, 200):
            sc = R.Scene(None, v, f, m, spatial_pct=sp, width=width, merge_leaves=merge,
                         max_leaf_size=2 if width == 4 else 4)
            infos[sp] = sc.info()
            assert infos[sp]["max_stack"] <= (96 if width == 4 else 44)
            assert sc.selfcheck(n, 23) == 0, (k, sp)
            sc.release()
        if k == 0:
            # the slivers' copies sit in more leaves; the cost falls by > 10%
            assert infos[10]["n_leaves"] > infos[-1]["n_leaves"]
            assert infos[10]["sah_cost"] < 0.9 * infos[-1]["sah_cost"]
            assert infos[200]["sah_cost"] <= infos[10]["sah_cost"] * 1.01


def test_host_bvh_spatial_splits_thread_independent(R):
    """The reference allowance passes down the tree by subtree size, so the
    tree does not depend on the number of build threads."""
    s = W.urban_block()
    infos = []
    for th in (1, 3, 8):
        sc = R.Scene(None, s.vertices, s.indices, s.tri_material, n_threads=th, spatial_pct=20)
        infos.append(sc.info())
        sc.release()
    for i in infos[1:]:
        for key in ("n_nodes", "n_leaves", "max_depth", "max_stack", "device_bytes", "sah_cost"):
            assert i[key] == infos[0][key], key


def test_bvh_option_validation(R):
    s = W.tiny_room()
    for bad in (dict(width=6), dict(width=8, max_leaf_size=5), dict(split_pct=201), dict(merge_leaves=3),
                dict(collapse=3), dict(spatial_pct=201), dict(spatial_pct=-2),
                dict(builder=2), dict(builder=1), dict(builder=1, width=8, max_leaf_size=2)):
        with pytest.raises(R.RadarError) as e:
            R.Scene(None, s.vertices, s.indices, s.tri_material, **bad)
        assert e.value.status == R.RR_EINVAL


def test_deep_median_fallback_bounds_depth(R):
    """A pathological mesh (triangles in a geometric progression along x)
    would give a very deep SAH tree; the builder caps inner depth below the
    traversal stack size."""
    n = 5000
    xs = np.cumsum(1.05 ** np.arange(n)) * 1e-3
    xs = np.minimum(xs, 1e6)
    V = np.zeros((3 * n, 3), np.float32)
    V[0::3, 0] = xs
    V[1::3, 0] = xs + 1e-3
    V[1::3, 1] = 0.5
    V[2::3, 0] = xs
    V[2::3, 2] = 0.5
    F = np.arange(3 * n, dtype=np.uint32).reshape(n, 3)
    for width, collapse in ((4, 1), (4, 2), (8, 0)):
        sc = R.Scene(None, V, F, np.zeros(n, np.uint16), max_leaf_size=1, width=width, collapse=collapse)
        assert sc.info()["max_stack"] <= (96 if width == 4 else 44)
        assert sc.selfcheck(3000, 11) == 0
        sc.release()


def test_postprocess_validation_without_device(R):
    """The epilogue checks its parameter block before it needs a context."""
    lib = R.load_library()
    good = R.make_post({})
    st = lib.rr_postprocess(None, None, 1, 1, 1, R.C.byref(good), None, None, None)
    assert st == R.RR_EINVAL and b"context" in lib.rr_last_error(None)
    for bad, word in ((dict(blur_sigma_bins=16.01), b"blur"), (dict(blur_sigma_bins=float("nan")), b"blur"),
                      (dict(uniform_amp=-1e-9), b"uniform"), (dict(perlin_amp=float("inf")), b"perlin"),
                      (dict(perlin_amp=1.0, perlin_cell_az=0.5), b"cell"), (dict(db_floor=0.0), b"db_floor"),
                      (dict(db_floor=float("-inf")), b"db_floor"), (dict(max_value=0), b"max_value"),
                      (dict(max_value=256), b"max_value")):
        pp = R.make_post(bad)
        st = lib.rr_postprocess(None, None, 1, 1, 1, R.C.byref(pp), None, None, None)
        assert st == R.RR_EINVAL and word in lib.rr_last_error(None), bad
    with pytest.raises(ValueError):
        R.make_post(dict(sigma=1.0))


def test_air_path_workspace_and_flags(R):
    """The air-path flag adds three 16-byte arrays with one entry per
    possible hit at depth >= 1, N_p (2 + 4 + ... + 2^(B-1)) (the visibility
    rays of every level); unknown flag bits are refused."""
    p = W.urban_block().params
    n = R.rr_workspace_query(p)
    na = R.rr_workspace_query(dict(p, flags=p["flags"] | R.RR_AIR_PATH))
    cap = 400 * 1024 * (2 + 4 + 8)
    assert 3 * 16 * cap <= na - n < 3 * 16 * cap + 1024
    with pytest.raises(R.RadarError) as e:
        R.rr_workspace_query(dict(p, flags=32))
    assert e.value.status == R.RR_EINVAL
