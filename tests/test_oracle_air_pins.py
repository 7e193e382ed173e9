"""Pins of the oracle's air-path (multi-path) returns (Sec. III-A, the
second return path) against an independent float64 model of small scenes of
flat quads written with numpy: nearest hits by a float64 ray/triangle solve,
mirror directions, the window fraction from the (separately pinned) window
coefficients, the receive gain of the arrival direction from its angle to the
beam axis, visibility of the sensor, and the range as half the round trip.
Plus the rules that have no geometry to model: no air return at depth 0
(the two paths coincide), none from inside a medium, and the energy ledger.
"""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

AIR = 16


def quad(c, u, v):
    c, u, v = (np.asarray(x, np.float64) for x in (c, u, v))
    p = [c - u - v, c + u - v, c + u + v, c - u + v]
    return [(p[0], p[1], p[2]), (p[0], p[2], p[3])]


def make_scene(quads, mats, params, pose=None):
    V, F, M = [], [], []
    for q, mi in quads:
        for tri in q:
            F.append([len(V), len(V) + 1, len(V) + 2])
            V.extend(tri)
            M.append(mi)
    return W.Scene("quads", np.array(V, np.float32), np.array(F, np.uint32), np.array(M, np.uint16), mats,
                   pose or W.identity_pose(), params)


def tri_hit(o, d, v0, v1, v2, tmax):
    """float64 ray/triangle solve: (t, smallest barycentric) or None."""
    A = np.column_stack([v1 - v0, v2 - v0, -d])
    if abs(np.linalg.det(A)) < 1e-14:
        return None
    u, v, t = np.linalg.solve(A, o - v0)
    if u < 0 or v < 0 or u + v > 1 or not (1e-9 < t <= tmax):
        return None
    return t, min(u, v, 1 - u - v)


def model_air(scene, orc, gain):
    """Per primary: first hit, mirror child, second hit, and the air-path
    return of the second hit.  Returns (image increment, set of uncertain
    bins, number of blocked returns)."""
    p = scene.params
    tris = [(scene.vertices[f].astype(np.float64)) for f in scene.indices]
    normals = []
    for v0, v1, v2 in tris:
        n = np.cross(v1 - v0, v2 - v0)
        normals.append(n / np.linalg.norm(n))
    S = np.asarray(scene.pose["position"], np.float64)
    axis = np.array([1.0, 0.0, 0.0])
    b = p["beam_width_rad"]
    sigma = (b / 2) / (math.sqrt(2) * __import__("scipy").special.erfinv(p["beam_prob"]))
    coeffs = [orc.window_coeffs(m, b) for m in scene.materials]

    def window(mi, c):
        k = coeffs[mi]
        w = k["a"] + k["beta"] * c + k["s"] * c ** scene.materials[mi]["C"]
        return min(max(w, 0.0), 1.0)

    def nearest(o, d, excl, tmax=np.inf):
        best = None
        for j, (v0, v1, v2) in enumerate(tris):
            if j == excl:
                continue
            h = tri_hit(o, d, v0, v1, v2, tmax)
            if h and (best is None or h[0] < best[0]):
                best = (h[0], j, h[1])
        return best

    img = np.zeros(p["n_bins"])
    uncertain, blocked = set(), 0
    per = {}  # primary -> (bin, energy) of its air-path return
    E0 = float(np.float32(1.0) / np.float32(p["rays_per_beam"]))
    for i in range(p["rays_per_beam"]):
        d = orc.primary(p, scene.pose, 0, i)["d"].astype(np.float64)
        r_max = p["n_bins"] * p["bin_size_m"]  # rays are traced up to this one-way path
        h1 = nearest(S, d, -1, r_max)
        if h1 is None:
            continue
        t1, j1, m1 = h1
        n = normals[j1]
        nf = n if d @ n < 0 else -n
        mi = int(scene.tri_material[j1])
        R1 = scene.materials[mi]["reflectance"]
        ci = -(d @ nf)
        E1 = E0 * R1 * (1 - window(mi, max(0.0, 2 * ci * ci - 1)))
        # the child leaves from the offset origin of the hit (pinned on its
        # own; it moves a 10 m point by some hundred ulps, 0.2 mm)
        p1 = orc.offset((S + t1 * d).astype(np.float32), nf.astype(np.float32)).astype(np.float64)
        d1 = d - 2 * (d @ nf) * nf
        d1 /= np.linalg.norm(d1)
        h2 = nearest(p1, d1, j1, r_max - t1)
        if h2 is None:
            continue
        t2, j2, m2 = h2
        n2 = normals[j2]
        nf2 = n2 if d1 @ n2 < 0 else -n2
        p2 = p1 + t2 * d1
        # the return leaves from the reflected child's offset origin (the
        # offset, pinned on its own, moves the point by some hundred ulps)
        po = orc.offset(p2.astype(np.float32), nf2.astype(np.float32)).astype(np.float64)
        v = S - po
        dist = np.linalg.norm(v)
        s = v / dist
        if s @ nf2 <= 0:
            continue
        mj = int(scene.tri_material[j2])
        R2 = scene.materials[mj]["reflectance"]
        r2 = d1 - 2 * (d1 @ nf2) * nf2
        r2 /= np.linalg.norm(r2)
        ci2 = -(d1 @ nf2)
        e_ret = E1 * R2 * window(mj, max(0.0, 2 * ci2 * ci2 - 1))
        e_air = min(E1 * R2 * window(mj, min(max(r2 @ s, 0.0), 1.0)), E1 * R2 - e_ret)
        g = 1.0
        if gain:
            w = po - S
            alpha = math.atan2(np.linalg.norm(np.cross(axis, w)), axis @ w)
            g = math.exp(-0.5 * (alpha / sigma) ** 2)
        q = (t1 + t2 + dist) / 2 / p["bin_size_m"]
        occ = nearest(po, s, j2, dist)
        # (float32 ranges carry a few ulp of 10 m: 5e-3 of a 4 mm bin)
        near = min(m1, m2) < 1e-6 or abs(q - round(q)) < 5e-3 or (occ is not None and occ[2] < 1e-6)
        if q >= p["n_bins"]:
            continue
        if near:
            uncertain.update({int(q) - 1, int(q), int(q) + 1})
        if occ is not None:
            blocked += 1
            per[i] = (int(q), 0.0, near)
            continue
        img[int(q)] += e_air * g
        per[i] = (int(q), e_air * g, near)
    model_air.per_primary = per
    return img, uncertain, blocked


GLOSSY = dict(kind=W.KIND_METAL, n=1.0, reflectance=0.6, A=0.2, B=0.3, C=20.0)


def mirror_floor(with_blocker=False, gain=True, seed=9, floor=None):
    beta = math.radians(3.0)
    nm = np.array([-math.cos(beta), 0.0, -math.sin(beta)])
    u = np.cross(nm, [0.0, 1.0, 0.0])
    u /= np.linalg.norm(u)
    quads = [(quad((10.0, 0.0, 0.0), 2.0 * u, (0.0, 2.0, 0.0)), 0),          # tilted metal mirror
             (quad((7.75, 0.0, -0.2), (1.75, 0.0, 0.0), (0.0, 2.0, 0.0)), 1)]  # Lambertian floor
    if with_blocker:
        quads.append((quad((6.0, 0.25, -0.165), (0.0, 0.25, 0.0), (0.0, 0.0, 0.025)), 1))
    params = W.sensor_params(1, 256, 2, 14000, bin_size_m=0.001, seed=seed,
                             flags=W.FLAG_BEAM_GAIN if gain else 0)
    return make_scene(quads, [W.material_metal(0.95), floor or W.material_lambertian(0.3)], params)


@pytest.mark.parametrize("gain", [False, True])
@pytest.mark.parametrize("blocker", [False, True])
@pytest.mark.parametrize("floor", ["lambertian", "glossy"])
def test_air_returns_match_float64_model(orc, gain, blocker, floor):
    """Tilted mirror 10 m ahead, floor 0.2 m below between it and the
    sensor: the mirror sends each primary down onto the floor, whose air-path
    return reaches the sensor ~1.5 degrees below the beam axis.  The glossy
    floor's window depends on the angle between its mirror direction and the
    direction to the sensor."""
    s = mirror_floor(with_blocker=blocker, gain=gain, floor=GLOSSY if floor == "glossy" else None)
    pa = dict(s.params, flags=s.params["flags"] | AIR)
    base = orc.scan_scene(s, records=True)
    air = orc.scan_scene(s, params=pa, records=True)
    # the hit records are those of the scan without air-path returns
    assert np.array_equal(base["records"], air["records"])
    diff = air["image"][0] - base["image"][0]
    want, unsure, n_blocked = model_air(s, orc, gain)
    per = model_air.per_primary
    assert want.sum() > 0 and len(per) > 200
    assert diff.sum() == pytest.approx(want.sum(), rel=1e-5)
    # primary by primary (masked scans): the bin and the energy of the return
    for i in range(0, 256, 11):
        if i not in per:
            continue
        mask = np.zeros(256, np.uint8)
        mask[i] = 1
        one = orc.scan_scene(s, params=pa, primary_mask=mask)["image"][0] - \
            orc.scan_scene(s, primary_mask=mask)["image"][0]
        b, e, near = per[i]
        if e == 0.0:
            assert not one.any(), i
        elif not near:
            assert np.nonzero(one)[0].tolist() == [b], i
            assert one[b] == pytest.approx(e, rel=1e-5), i
    outcomes = air["air_records"]
    assert int((outcomes == 1).sum()) == n_blocked
    if blocker:
        assert n_blocked > 10
    else:
        assert n_blocked == 0
    # gain on: the returns arrive ~1.5 degrees off the beam axis
    if gain:
        plain = model_air(s, orc, False)[0]
        assert 0.05 < want.sum() / plain.sum() < 0.6


def test_no_air_return_at_depth_zero(orc):
    """A plane facing the sensor: every hit is a primary hit, whose path back
    to the sensor is the retrace path itself."""
    s = W.plane_scene(3.0, W.material_lambertian(0.5), n_azimuth=8, rays_per_beam=64, max_bounces=3,
                      n_bins=200, bin_size_m=0.044)
    a = orc.scan_scene(s, records=True)
    b = orc.scan_scene(s, params=dict(s.params, flags=s.params["flags"] | AIR), records=True)
    assert np.array_equal(a["image"], b["image"])
    assert (b["air_records"] == -2).all()


def test_no_air_return_from_inside_a_medium(orc):
    """Slab: the back-face hit happens inside the material (no air return);
    its path to the sensor would cross the front face, which the ledger
    would show as blocked energy."""
    s = W.slab_scene(2.0, 0.05, W.material_dielectric(2.5, roughness=0.3), n_azimuth=4, rays_per_beam=64,
                     max_bounces=3, n_bins=256, bin_size_m=0.044)
    a = orc.scan_scene(s)
    b = orc.scan_scene(s, params=dict(s.params, flags=s.params["flags"] | AIR), records=True)
    assert np.array_equal(a["image"], b["image"])
    e = dict(zip(orc.E_SLOTS, b["energy"].sum(axis=0)))
    assert e["blocked"] == 0.0
    assert (b["air_records"][:, 1] == -2).all()  # heap 2..3: depth-1 segments
    assert (b["air_records"][:, 2] == -2).all()


def test_air_energy_ledger_closes(orc):
    s = W.tiny_room()
    out = orc.scan_scene(s, params=dict(s.params, flags=s.params["flags"] | AIR), threads=8)
    en = out["energy"]
    assert np.allclose(en[:, 0], en[:, 1:].sum(axis=1), rtol=0, atol=1e-12)
    e = dict(zip(orc.E_SLOTS, en.sum(axis=0)))
    assert e["blocked"] > 0 and e["returned_in"] > 0


def test_air_translation_invariance(orc):
    s = W.tiny_room(n_azimuth=40, rays_per_beam=16)
    p = dict(s.params, flags=s.params["flags"] | AIR)
    a = orc.scan_scene(s, params=p)["image"]
    t = W.transform_scene(s, shift=(0.5, -0.25, 0.125))
    b = orc.scan_scene(t, params=p)["image"]
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-4
