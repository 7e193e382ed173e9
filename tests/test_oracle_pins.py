"""Pins of the CPU oracle against things other than itself: numpy's Philox,
scipy's erfinv, Gamma and quadrature, scipy's rotations, a float64 linear
solve, Fresnel's sine/tangent form, closed-form scenes and symmetries.

Each pin is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign or index, a swapped operand) fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, special, stats
from scipy.spatial.transform import Rotation

import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def numpy_philox(key, ctr):
    """numpy increments the 256-bit counter before producing a block, so the
    block for counter c is the first one after setting c - 1."""
    c = [int(x) for x in ctr]
    v = (c[0] | (c[1] << 64) | (c[2] << 128) | (c[3] << 192)) - 1
    v %= 1 << 256
    prev = np.array([(v >> (64 * j)) & ((1 << 64) - 1) for j in range(4)], dtype=np.uint64)
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=prev)
    return [int(x) for x in g.random_raw(4)]


# ----------------------------------------------------------------- RNG
def test_philox_known_answer(orc):
    # published known-answer vector of Philox4x64-10 (Salmon et al., SC'11,
    # Random123 kat file): counter 0, key 0
    assert orc.philox4x64_10([0, 0], [0, 0, 0, 0]) == [
        0x16554D9ECA36314C, 0xDB20FE9D672D0FDC, 0xD7E772CEE186176B, 0x7E68B68AEC7BA23B]


@pytest.mark.parametrize("key,ctr", [
    ((0x5EED, 0), (0, 0, 0, 0)), ((0x5EED, 7), (399, 63, 0, 0)),
    ((2**64 - 1, 12345), (2**40 + 3, 2**20 - 1, 0, 0)), ((1, 2), (2**64 - 1, 5, 0, 0)),
])
def test_philox_matches_numpy(orc, key, ctr):
    assert orc.philox4x64_10(key, ctr) == numpy_philox(key, ctr)


# ----------------------------------------------------------------- Eq. 2
def test_erfinv_and_sigma(orc):
    c = GOLD["d3_radius_scale"]
    assert orc.erfinv(0.9) == pytest.approx(special.erfinv(0.9), rel=1e-15, abs=0)
    assert orc.erfinv(0.9) == pytest.approx(c["erfinv_0_9"], rel=2e-16)
    for p in (0.1, 0.5, 0.75, 0.99, 0.999999):
        assert orc.erfinv(p) == pytest.approx(special.erfinv(p), rel=1e-14)
    assert math.degrees(orc.sigma_r(math.radians(10.0), 0.9)) == pytest.approx(c["sigma_r_deg_b10"], rel=1e-7)
    assert math.degrees(orc.sigma_r(math.radians(2.0), 0.9)) == pytest.approx(c["sigma_r_deg_b2"], rel=1e-7)


def _angle_from_axis(d, phi):
    axis = np.array([math.cos(phi), math.sin(phi), 0.0])
    return math.acos(min(1.0, float(np.dot(d.astype(np.float64), axis))))


def test_d3_cone_statistics(orc):
    """P(angular offset <= b/2) = P (Eq. 2), mean receive gain -> 1/sqrt 2,
    polar angle omega uniform, computed from the returned directions."""
    b = math.radians(2.0)
    prm = W.sensor_params(360, 64, 1, 16, beam_width_deg=2.0, seed=99)
    pose = W.identity_pose()
    n = 0
    inside, gs, om = 0, [], []
    for k in range(0, 360, 3):
        phi = 2 * math.pi * k / 360
        for i in range(64):
            p = orc.primary(prm, pose, k, i)
            a = _angle_from_axis(p["d"], phi)
            inside += a <= b / 2
            gs.append(float(p["g"]))
            d = p["d"].astype(np.float64)
            inc = math.asin(d[2])
            az = math.atan2(d[1], d[0]) - phi
            az = (az + math.pi) % (2 * math.pi) - math.pi
            if math.hypot(az, inc) > 1e-6:
                om.append(math.atan2(inc, az))
            n += 1
    frac = inside / n
    assert abs(frac - 0.9) < 5 * math.sqrt(0.09 / n)
    g = np.array(gs)
    assert abs(g.mean() - 1 / math.sqrt(2)) < 5 * g.std() / math.sqrt(n)
    assert stats.kstest((np.array(om) + math.pi) / (2 * math.pi), "uniform").pvalue > 1e-3


def test_primary_gain_from_numpy_philox(orc):
    """The receive gain exp(-z^2/2) with z from Box-Muller on numpy's Philox
    stream (key = (seed, scan_id), counter = (k, i, 0, 0))."""
    prm = W.sensor_params(16, 8, 1, 16, seed=0xABCDEF, scan_id=3)
    for k, i in [(0, 0), (5, 7), (15, 3)]:
        x = numpy_philox((0xABCDEF, 3), (k, i, 0, 0))
        u1 = ((x[0] >> 11) + 1) * 2.0 ** -53
        u2 = (x[1] >> 11) * 2.0 ** -53
        z = math.sqrt(-2 * math.log(u1)) * math.cos(2 * math.pi * u2)
        p = orc.primary(prm, W.identity_pose(), k, i)
        assert p["z"] == pytest.approx(z, rel=1e-12, abs=1e-12)
        assert float(p["g"]) == np.float32(math.exp(-z * z / 2))


def test_zero_width_beam_direction_uses_pose_rotation(orc):
    quat = np.array([0.9, 0.1, -0.3, 0.2])
    quat /= np.linalg.norm(quat)
    pose = dict(position=(1.0, -2.0, 0.5), quat_wxyz=tuple(quat))
    prm = W.sensor_params(12, 2, 1, 16, beam_width_rad=0.0)
    rot = Rotation.from_quat([quat[1], quat[2], quat[3], quat[0]])
    for k in range(12):
        phi = 2 * math.pi * k / 12
        p = orc.primary(prm, pose, k, 1)
        want = rot.apply([math.cos(phi), math.sin(phi), 0.0])
        np.testing.assert_allclose(p["d"], want, atol=1e-7)
        np.testing.assert_array_equal(p["o"], np.float32([1.0, -2.0, 0.5]))


def test_fixed_pattern_and_mirror_pairs(orc):
    prm = W.sensor_params(8, 6, 1, 16, flags=W.FLAG_FIXED_PATTERN | W.FLAG_MIRROR_PAIRS)
    pose = W.identity_pose()
    for k in (0, 3):
        phi = 2 * math.pi * k / 8
        for i in (0, 2, 4):
            a = orc.primary(prm, pose, k, i)["d"].astype(np.float64)
            b = orc.primary(prm, pose, k, i + 1)["d"].astype(np.float64)
            # same inclination, azimuth offset mirrored about the beam axis
            assert a[2] == b[2]
            off_a = math.atan2(a[1], a[0]) - phi
            off_b = math.atan2(b[1], b[0]) - phi
            assert off_a == pytest.approx(-off_b, abs=1e-6)
    d0 = orc.primary(prm, pose, 0, 4)["d"].astype(np.float64)
    d3 = orc.primary(prm, pose, 3, 4)["d"].astype(np.float64)
    r3 = Rotation.from_euler("z", 2 * math.pi * 3 / 8).apply(d0)
    np.testing.assert_allclose(d3, r3, atol=1e-6)


# ----------------------------------------------------------------- geometry
def test_moller_trumbore_hand_cases(orc):
    # axis-aligned triangle in the plane x = 3: t = 3 exactly
    v0, v1, v2 = (3.0, -1.0, -1.0), (3.0, 2.0, -1.0), (3.0, -1.0, 2.0)
    assert orc.ray_triangle((0, 0, 0), (1, 0, 0), v0, v1, v2) == 3.0
    assert orc.ray_triangle((0, 0, 0), (-1, 0, 0), v0, v1, v2) is None   # behind
    assert orc.ray_triangle((0, 0, 0), (1, 0, 0), v0, v1, v2, tmax=2.5) is None
    assert orc.ray_triangle((0, 0, 0), (1, 0, 0), v0, v1, v2, tmax=3.0) == 3.0
    assert orc.ray_triangle((0, 5, 0), (1, 0, 0), v0, v1, v2) is None     # outside
    assert orc.ray_triangle((0, 0, 0), (0, 1, 0), v0, v1, v2) is None     # parallel
    # both faces are hit
    assert orc.ray_triangle((6, 0, 0), (-1, 0, 0), v0, v1, v2) == 3.0


def test_moller_trumbore_vs_float64_solve(orc):
    rng = np.random.default_rng(5)
    agree = 0
    for _ in range(600):
        v = rng.normal(size=(3, 3)) * 2 + np.array([4.0, 0, 0])
        o = rng.normal(size=3) * 0.2
        d = rng.normal(size=3) + np.array([2.0, 0, 0])
        d /= np.linalg.norm(d)
        v32, o32, d32 = v.astype(np.float32), o.astype(np.float32), d.astype(np.float32)
        V, O, D = v32.astype(np.float64), o32.astype(np.float64), d32.astype(np.float64)
        M = np.column_stack([-D, V[1] - V[0], V[2] - V[0]])
        t, u, w = np.linalg.solve(M, O - V[0])
        margin = min(u, w, 1 - u - w)
        got = orc.ray_triangle(o32, d32, *v32)
        if abs(margin) < 1e-4 or abs(t) < 1e-4:
            continue
        inside = margin > 0 and t > 0
        assert (got is not None) == inside
        if inside:
            assert got == pytest.approx(t, rel=2e-5)
        agree += 1
    assert agree > 500


def test_offset_moves_origin_off_the_surface(orc):
    rng = np.random.default_rng(2)
    for scale in (1e-3, 0.02, 1.0, 40.0, 700.0):
        for _ in range(50):
            p = (rng.normal(size=3) * scale).astype(np.float32)
            n = rng.normal(size=3)
            n = (n / np.linalg.norm(n)).astype(np.float32)
            q = orc.offset(p, n)
            dp = q.astype(np.float64) - p.astype(np.float64)
            assert float(np.dot(dp, n.astype(np.float64))) > 0.0
            assert np.linalg.norm(dp) < 1e-4 * max(1.0, float(np.abs(p).max()))


def _steps_along(p: np.float32, k: int) -> np.float32:
    """p moved |k| representable float32 values towards sign(k) * inf."""
    target = np.float32(np.inf) if k > 0 else np.float32(-np.inf)
    for _ in range(abs(k)):
        p = np.nextafter(p, target, dtype=np.float32)
    return p


def test_offset_ulp_distance_and_published_constants(orc):
    """Waechter & Binder (Ray Tracing Gems, 2019, ch. 6): away from the origin
    (|p_i| >= 1/32) the coordinate moves by trunc(256 n_i) representable
    float32 values in the direction of n_i; closer to it, by the distance
    n_i / 65536.  The steps are counted with nextafter, not with the bit
    arithmetic the oracle uses, and the coordinates are chosen on both sides
    of 1/32 and 1/16 so that another int scale (128), float scale (1/32768)
    or origin threshold (1/16) fails here."""
    rng = np.random.default_rng(17)
    mags = [1.0 / 64, 0.02, 1.0 / 32, 0.04, 0.0625, 0.09, 0.7, 1.0, 3.0, 255.9, 4096.0, 1e6]
    checked_ulp = checked_near = 0
    for m in mags:
        for sign in (1.0, -1.0):
            for _ in range(6):
                p = np.array([sign * m * rng.uniform(1.0, 1.2) if m not in (1.0 / 32,) else sign * m,
                              -sign * m * rng.uniform(1.0, 1.2), sign * m], dtype=np.float32)
                n = rng.normal(size=3)
                n = (n / np.linalg.norm(n)).astype(np.float32)
                q = orc.offset(p, n)
                for i in range(3):
                    if abs(float(p[i])) >= 1.0 / 32:
                        k = int(np.trunc(np.float32(256.0) * n[i]))
                        want = _steps_along(p[i], k)
                        checked_ulp += 1
                    else:
                        want = np.float32(p[i] + np.float32(n[i] / np.float32(65536.0)))
                        checked_near += 1
                    assert q[i] == want, (float(p[i]), float(n[i]), float(q[i]), float(want))
    assert checked_ulp > 150 and checked_near > 40
    # an axis-aligned normal at 1/32 exactly: 256 steps, the ulp form
    p = np.array([1.0 / 32, 0.5, -2.0], dtype=np.float32)
    q = orc.offset(p, np.array([1.0, 0.0, 0.0], dtype=np.float32))
    assert q[0] == _steps_along(np.float32(1.0 / 32), 256)
    assert q[1] == p[1] and q[2] == p[2]


# ----------------------------------------------------------------- Snell / Fresnel
def _dir_at(theta):
    """unit direction hitting the plane with normal (-1,0,0) at incidence theta"""
    return np.array([math.cos(theta), math.sin(theta), 0.0], dtype=np.float32)


NG_FACING = np.array([-1.0, 0.0, 0.0], dtype=np.float32)


@pytest.mark.parametrize("n", [1.5, 2.0, 2.5, 6.0])
def test_fresnel_normal_incidence(orc, n):
    m = W.material_dielectric(n)
    r = orc.interact((1, 0, 0), NG_FACING, m, 0.0, 1.0, W.FLAG_RETURN_ALL)
    assert r["entering"] and r["has_refract"] and not r["tir"]
    assert r["R"] == pytest.approx(GOLD["fresnel_normal_incidence"][str(n)], rel=1e-12)
    assert r["R"] + r["T"] == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_allclose(r["refl"], [-1, 0, 0], atol=0)
    np.testing.assert_allclose(r["refr"], [1, 0, 0], atol=0)
    # leaving the medium: the same reflectance (reciprocity at normal incidence)
    out = orc.interact((1, 0, 0), -NG_FACING, m, 0.0, np.float32(n), W.FLAG_RETURN_ALL)
    assert not out["entering"]
    assert out["R"] == pytest.approx(r["R"], rel=1e-6)


@pytest.mark.parametrize("n", [1.5, 2.0, 2.5, 6.0])
def test_snell_and_fresnel_sine_tangent_form(orc, n):
    """Snell n1 sin t1 = n2 sin t2, unit directions, coplanarity, and the
    reflectance against Fresnel's sine/tangent form of the equations."""
    m = W.material_dielectric(n)
    for deg in (5.0, 20.0, 40.0, 60.0, 80.0, 89.0):
        th = math.radians(deg)
        d = _dir_at(th)
        r = orc.interact(d, NG_FACING, m, 0.0, 1.0, W.FLAG_RETURN_ALL)
        t = r["refr"].astype(np.float64)
        rf = r["refl"].astype(np.float64)
        assert np.linalg.norm(t) == pytest.approx(1.0, abs=1e-6)
        assert np.linalg.norm(rf) == pytest.approx(1.0, abs=1e-6)
        assert abs(t[2]) < 1e-7 and abs(rf[2]) < 1e-7           # plane of incidence
        ti = math.asin(min(1.0, abs(float(d[1]))))
        tt = math.asin(abs(t[1]))
        assert 1.0 * math.sin(ti) == pytest.approx(n * math.sin(tt), abs=2e-6)
        assert math.asin(abs(rf[1])) == pytest.approx(ti, abs=2e-6)  # mirror angle
        assert rf[0] < 0 and t[0] > 0
        rs = -math.sin(ti - tt) / math.sin(ti + tt)
        rp = math.tan(ti - tt) / math.tan(ti + tt)
        assert r["R"] == pytest.approx(0.5 * (rs * rs + rp * rp), rel=2e-5, abs=1e-7)
        # reciprocity: coming back along the refracted ray from inside
        back = orc.interact(-t.astype(np.float32), -NG_FACING * -1, m, 0.0, np.float32(n),
                            W.FLAG_RETURN_ALL)
        assert back["R"] == pytest.approx(r["R"], rel=1e-4, abs=1e-6)


@pytest.mark.parametrize("n", [1.5, 2.0, 6.0])
def test_total_internal_reflection_threshold(orc, n):
    crit = math.radians(GOLD["critical_angle_deg"][str(n)])
    m = W.material_dielectric(n)
    for delta, tir in ((-2e-3, False), (2e-3, True)):
        th = crit + delta
        d = np.array([math.cos(th), math.sin(th), 0.0], dtype=np.float32)
        # inside the medium heading out through a face whose normal is +x
        r = orc.interact(d, np.float32([1, 0, 0]), m, 0.0, np.float32(n), W.FLAG_RETURN_ALL)
        assert not r["entering"]
        assert r["tir"] == tir
        if tir:
            assert r["R"] == 1.0 and r["T"] == 0.0 and not r["has_refract"]
        else:
            assert r["R"] < 1.0 and r["has_refract"]


def test_brewster_angle(orc):
    n = 2.5
    tb = math.atan(n)
    d = _dir_at(tb)
    r = orc.interact(d, NG_FACING, W.material_dielectric(n), 0.0, 1.0, W.FLAG_RETURN_ALL)
    # reflected and refracted rays are perpendicular; only s-polarised light reflects
    assert abs(float(np.dot(r["refl"].astype(np.float64), r["refr"].astype(np.float64)))) < 2e-6
    ct = math.cos(math.asin(math.sin(tb) / n))
    rs = (math.cos(tb) - n * ct) / (math.cos(tb) + n * ct)
    assert r["R"] == pytest.approx(rs * rs / 2, rel=1e-5)


def test_metal_and_lambertian_split(orc):
    d = _dir_at(0.3)
    for m in (W.material_metal(0.95), W.material_lambertian(0.3)):
        r = orc.interact(d, NG_FACING, m, math.radians(2), 1.0, 0)
        assert r["R"] == pytest.approx(m["reflectance"], rel=1e-7)
        assert r["T"] == 0.0 and not r["has_refract"]


# ----------------------------------------------------------------- BRDF window (Eq. 3-5)
def test_lobe_integral_gamma_closed_form(orc):
    for c, v in GOLD["lobe_integral"].items():
        if c.startswith("_"):
            continue
        C = float(c)
        gam = math.sqrt(math.pi) * math.exp(special.gammaln((C + 1) / 2) - special.gammaln(C / 2 + 1))
        assert orc.lobe_integral(C) == pytest.approx(gam, rel=1e-10)
        assert orc.lobe_integral(C) == pytest.approx(v, rel=1e-10)


def test_window_against_quadrature(orc):
    """w(omega) = integral over [omega - b/2, omega + b/2] of the normalised
    lobe; the A and B parts are exact, the S part converges as b -> 0."""
    b = math.radians(2.0)
    # pure B lobe: (1/2) * integral of cos over the window
    wc = orc.window_coeffs(dict(kind=0, n=1.5, reflectance=0, A=0.0, B=1.0, C=5.0), b)
    for om in (0.0, 0.3, 1.0):
        q = integrate.quad(math.cos, om - b / 2, om + b / 2)[0] / 2.0
        assert wc["beta"] * math.cos(om) == pytest.approx(q, rel=1e-12)
    # Lambertian: b / pi at any angle
    wl = orc.window_coeffs(W.material_lambertian(0.3), b)
    assert wl["a"] == pytest.approx(b / math.pi, rel=1e-14)
    assert wl["beta"] == 0 and wl["s"] == 0
    # mixed lobe, narrow window: midpoint rule ~ exact integral
    m = dict(kind=0, n=1.5, reflectance=0, A=0.2, B=0.3, C=30.0)
    bs = math.radians(0.1)
    wm = orc.window_coeffs(m, bs)
    A32, B32 = float(np.float32(0.2)), float(np.float32(0.3))
    Z = A32 * math.pi + 2 * B32 + (1 - A32 - B32) * GOLD["lobe_integral"]["30"]
    assert wm["Z"] == pytest.approx(Z, rel=1e-10)
    for om in (0.0, 0.2):
        f = lambda a: 0.2 + 0.3 * math.cos(a) + 0.5 * math.cos(a) ** 30
        q = integrate.quad(f, om - bs / 2, om + bs / 2)[0] / Z
        c = math.cos(om)
        assert wm["a"] + wm["beta"] * c + wm["s"] * c ** 30 == pytest.approx(q, rel=1e-5)


def test_smooth_lobe_peak_return(orc):
    # C = 2000, b = 2 deg, normal incidence: w = b / I(2000) = 0.6228
    r = orc.interact((1, 0, 0), NG_FACING, W.material_metal(0.95), math.radians(2.0), 1.0, 0)
    b32 = float(np.float32(math.radians(2.0)))   # the beam width travels as float32
    assert r["w"] == pytest.approx(b32 / GOLD["lobe_integral"]["2000"], rel=1e-9)
    assert r["w"] == pytest.approx(0.6228, abs=1e-4)
    # at 50 degrees incidence the mirror lobe points far from the sensor: 0
    r = orc.interact(_dir_at(math.radians(50)), NG_FACING, W.material_metal(0.95),
                     math.radians(2.0), 1.0, 0)
    assert r["w"] == 0.0


# ----------------------------------------------------------------- scenes with closed forms
def _gains_from_numpy(seed, scan_id, k, n_s):
    g = []
    for i in range(n_s):
        x = numpy_philox((seed, scan_id), (k, i, 0, 0))
        u1 = ((x[0] >> 11) + 1) * 2.0 ** -53
        u2 = (x[1] >> 11) * 2.0 ** -53
        z = math.sqrt(-2 * math.log(u1)) * math.cos(2 * math.pi * u2)
        g.append(float(np.float32(math.exp(-z * z / 2))))
    return np.array(g)


def test_plane_at_bin_centre(orc):
    dr = 0.044
    dist = 100.5 * dr
    s = W.plane_scene(dist, W.material_lambertian(0.3), n_azimuth=1, rays_per_beam=256,
                      max_bounces=1, n_bins=1024, bin_size_m=dr, seed=77)
    out = orc.scan_scene(s)
    img = out["image"][0]
    assert np.nonzero(img)[0].tolist() == [100]
    b = math.radians(2.0)
    E0 = float(np.float32(1.0) / np.float32(256))
    g = _gains_from_numpy(77, 0, 0, 256)
    assert img[100] == pytest.approx(0.3 * (b / math.pi) * E0 * g.sum(), rel=1e-6)


def test_slab_front_and_back_returns(orc):
    dr, d, h, n = 0.044, 2.0, 0.05, 2.5
    s = W.slab_scene(d, h, W.material_dielectric(n), n_azimuth=1, rays_per_beam=64,
                     max_bounces=3, n_bins=256, bin_size_m=dr, beam_width_rad=0.0,
                     flags=W.FLAG_RETURN_ALL)
    s.pose = W.identity_pose((0.0, 0.31, 0.17))
    out = orc.scan_scene(s)
    img = out["image"][0]
    R = GOLD["fresnel_normal_incidence"]["2.5"]
    front, back = int(d / dr), int((d + n * h) / dr)
    assert (front, back) == (45, 48)
    assert np.nonzero(img)[0].tolist() == [front, back]
    E = 64 * float(np.float32(1.0) / np.float32(64))
    assert img[front] == pytest.approx(E * R, rel=1e-6)
    assert img[back] == pytest.approx(E * (1 - R) * R, rel=1e-6)
    e = dict(zip(__import__("oracle").E_SLOTS, out["energy"][0]))
    assert e["escaped"] == pytest.approx(E * (1 - R) ** 2, rel=1e-6)
    assert e["absorbed"] == pytest.approx(0.0, abs=1e-15)


def test_lidar_like_empty_room(orc):
    """b = 0, one bounce, every hit returned: column k's only return is at
    the wall distance min(5/|cos phi|, 4/|sin phi|) with the wall albedo."""
    dr, naz = 0.044, 400
    s = W.empty_room(0.3, n_azimuth=naz, rays_per_beam=4, max_bounces=1, n_bins=1024,
                     bin_size_m=dr, beam_width_rad=0.0, flags=W.FLAG_RETURN_ALL)
    out = orc.scan_scene(s)
    checked = 0
    for k in range(naz):
        phi = 2 * math.pi * k / naz
        c, sn = abs(math.cos(phi)), abs(math.sin(phi))
        rho = min(5 / c if c > 1e-12 else np.inf, 4 / sn if sn > 1e-12 else np.inf)
        q = rho / dr
        if abs(q - round(q)) < 1e-3:
            continue
        nz = np.nonzero(out["image"][k])[0].tolist()
        assert nz == [int(q)], k
        assert out["image"][k][int(q)] == pytest.approx(0.3, rel=1e-6)
        checked += 1
    assert checked > 390


def test_closest_hit_matches_float64_brute_force(orc):
    """Primary hits of the tiny room against a float64 linear-solve brute
    force written here (every triangle, nearest t)."""
    s = W.tiny_room(n_azimuth=40, rays_per_beam=8, max_bounces=1)
    out = orc.scan_scene(s, records=True, exempt=True)
    V = s.vertices.astype(np.float64)
    F = s.indices.astype(np.int64)
    n_ok = 0
    for k in range(40):
        for i in range(8):
            p = orc.primary(s.params, s.pose, k, i)
            O, D = p["o"].astype(np.float64), p["d"].astype(np.float64)
            best, bt = -1, np.inf
            for j, f in enumerate(F):
                M = np.column_stack([-D, V[f[1]] - V[f[0]], V[f[2]] - V[f[0]]])
                if abs(np.linalg.det(M)) < 1e-12:
                    continue
                t, u, w = np.linalg.solve(M, O - V[f[0]])
                if t > 0 and u >= 0 and w >= 0 and u + w <= 1 and t < bt:
                    best, bt = j, t
            lp = k * 8 + i
            if out["exempt"][lp]:
                continue
            assert out["records"][lp, 0] == best
            n_ok += 1
    assert n_ok > 300


def test_records_heap_layout(orc):
    """One dielectric triangle facing the sensor (normal -x): the primary hits
    it (heap 1); its reflected
    child (heap 2) and refracted child (heap 3) miss; nothing deeper."""
    m = W.material_dielectric(2.0)
    s = W.single_triangle_scene((3, -2, -2), (3, 0, 3), (3, 2, -2), m, n_azimuth=1,
                                rays_per_beam=4, max_bounces=3, n_bins=256)
    out = orc.scan_scene(s, records=True)
    for r in out["records"]:
        assert r.tolist() == [0, -1, -1, -2, -2, -2, -2]
    sm = W.single_triangle_scene((3, -2, -2), (3, 0, 3), (3, 2, -2), W.material_metal(0.95),
                                 n_azimuth=1, rays_per_beam=4, max_bounces=2, n_bins=256)
    for r in orc.scan_scene(sm, records=True)["records"]:
        assert r.tolist() == [0, -1, -2]


def test_degenerate_triangle_is_never_hit(orc):
    # zero-area triangle straddling the beam in front of a plane at x = 4
    V = np.array([[2, -1, 0], [2, 1, 0], [2, 0, 0],
                  [4, -5, -5], [4, 5, -5], [4, 5, 5], [4, -5, 5]], dtype=np.float32)
    F = np.array([[0, 1, 2], [3, 5, 4], [3, 6, 5]], dtype=np.uint32)
    M = np.zeros(3, dtype=np.uint16)
    prm = W.sensor_params(1, 8, 1, 256, beam_width_rad=0.0)
    out = orc.scan(V, F, M, W.identity_pose((0, 0, 0)), prm, [W.material_lambertian(0.5)],
                   records=True)
    assert set(out["records"][:, 0].tolist()) <= {1, 2}


# ----------------------------------------------------------------- invariants
def test_energy_conservation_tiny_room(orc):
    s = W.tiny_room()
    e = orc.scan_scene(s)["energy"]
    E0 = 64 * float(np.float32(1) / np.float32(64))
    np.testing.assert_allclose(e[:, 0], E0, rtol=1e-15)
    np.testing.assert_allclose(e[:, 1:].sum(1), e[:, 0], rtol=0, atol=1e-12)
    assert (e >= -1e-18).all()


def test_lossless_dielectric_absorbs_nothing(orc):
    s = W.urban_block()
    cols = [0, 133, 277]
    s.params = dict(s.params, rays_per_beam=8)
    e = orc.scan_scene(s, columns=cols)["energy"]
    assert np.abs(e[:, 4]).max() < 1e-15
    np.testing.assert_allclose(e[:, 1:].sum(1), e[:, 0], rtol=0, atol=1e-12)


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_mirror_symmetry(orc):
    s = W.mirror_scene(flags=W.FLAG_BEAM_GAIN | W.FLAG_FIXED_PATTERN | W.FLAG_MIRROR_PAIRS)
    img = orc.scan_scene(s)["image"]
    nz = s.params["n_azimuth"]
    mirrored = img[[(nz - k) % nz for k in range(nz)]]
    assert img.sum() > 0
    assert _rel_l2(img, mirrored) < 1e-6


def test_rotation_shifts_columns(orc):
    s = W.tiny_room(n_azimuth=64, rays_per_beam=32, flags=W.FLAG_BEAM_GAIN | W.FLAG_FIXED_PATTERN)
    r = W.transform_scene(s, yaw=2 * math.pi / 64)
    a = orc.scan_scene(s)["image"]
    b = orc.scan_scene(r)["image"]
    assert _rel_l2(b[1:], a[:-1]) < 1e-3
    assert _rel_l2(b[0], a[-1]) < 1e-3


def test_translation_invariance(orc):
    s = W.tiny_room(n_azimuth=64, rays_per_beam=32)
    t = W.transform_scene(s, shift=(8.0, -4.0, 2.0))
    a = orc.scan_scene(s)["image"]
    b = orc.scan_scene(t)["image"]
    # re-rounded float32 vertices move single returns across a bin edge, so
    # compare column totals and profiles smoothed over neighbouring bins
    np.testing.assert_allclose(b.sum(1), a.sum(1), rtol=2e-3, atol=1e-9)
    k = np.ones(3)
    sa = np.array([np.convolve(r, k, "same") for r in a])
    sb = np.array([np.convolve(r, k, "same") for r in b])
    assert _rel_l2(sb, sa) < 2e-2


def test_retrace_return_angle(orc):
    """The return travels back along the incoming ray, so the lobe is read at
    the angle between the mirror direction and -d (measured here from the
    returned directions) and integrated over the beam window (Eq. 4)."""
    b = math.radians(3.0)
    b32 = float(np.float32(b))
    m = dict(kind=1, n=1.0, reflectance=1.0, A=0.0, B=1.0, C=4.0)   # pure B lobe, Z = 2
    for deg in (0.0, 10.0, 20.0, 33.0, 44.0):
        d = _dir_at(math.radians(deg))
        r = orc.interact(d, NG_FACING, m, b, 1.0, 0)
        back = -d.astype(np.float64)
        om = math.acos(min(1.0, float(np.dot(r["refl"].astype(np.float64), back))))
        want = integrate.quad(math.cos, om - b32 / 2, om + b32 / 2)[0] / 2.0
        assert r["w"] == pytest.approx(want, rel=1e-5, abs=1e-9), deg
