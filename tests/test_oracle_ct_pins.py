"""Pins of the oracle's Cook-Torrance material kind (the user-defined BRDF of
the experiments, Sec. IV; Cook & Torrance 1982 with the GGX distribution and
Smith masking of Walter et al. 2007) and of the elliptic beam stretch
(Sec. III-A): each term against an independent form (GGX normalisation by
quadrature, GGX in its tangent form, Smith masking in its Lambda form,
Fresnel in its sine/tangent form), the assembled BRDF against those, its
reciprocity and energy bound, a plane whose returns follow in closed form,
and the stretch against the unstretched cone."""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


def sph(theta, phi):
    return np.array([math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi), math.cos(theta)])


@pytest.mark.parametrize("alpha", [0.1, 0.3, 0.5, 1.0])
def test_ggx_distribution_is_normalised(orc, alpha):
    """The projected microfacet area integrates to one over the hemisphere."""
    m = W.material_cook_torrance(0.0, alpha, 1.5, 0.0)
    n = (0.0, 0.0, 1.0)

    def dcos(theta):
        h = sph(theta, 0.0)
        return orc.ct_terms(m, n, h, h)[0] * math.cos(theta) * math.sin(theta)

    val, _ = integrate.quad(dcos, 0.0, math.pi / 2, limit=400, epsabs=1e-12)
    assert 2 * math.pi * val == pytest.approx(1.0, abs=2e-6)


def fresnel_sine_tangent(n, cos_i):
    ti = math.acos(min(1.0, cos_i))
    if ti == 0.0:
        return ((n - 1) / (n + 1)) ** 2
    tt = math.asin(math.sin(ti) / n)
    rs = math.sin(ti - tt) / math.sin(ti + tt)
    rp = math.tan(ti - tt) / math.tan(ti + tt)
    return 0.5 * (rs * rs + rp * rp)


def reference_f(kd, alpha, n_idx, n, l, v):
    """The same BRDF from independent forms of its terms."""
    nl, nv = n @ l, n @ v
    h = unit(l + v)
    th = math.acos(min(1.0, n @ h))
    D = alpha ** 2 / (math.pi * math.cos(th) ** 4 * (alpha ** 2 + math.tan(th) ** 2) ** 2)

    def G1(x):
        t2 = (1 - x * x) / (x * x)
        lam = (-1 + math.sqrt(1 + alpha ** 2 * t2)) / 2
        return 1 / (1 + lam)

    F = fresnel_sine_tangent(n_idx, v @ h)
    return kd / math.pi + (1 - kd) * D * F * G1(nl) * G1(nv) / (4 * nl * nv)


def test_brdf_against_independent_terms(orc):
    rng = np.random.default_rng(4)
    n = np.array([0.0, 0.0, 1.0])
    for _ in range(300):
        kd, alpha, n_idx = rng.uniform(0, 1), rng.uniform(0.05, 1.0), rng.uniform(1.2, 100.0)
        l = unit(sph(rng.uniform(0, 1.45), rng.uniform(0, 2 * math.pi)))
        v = unit(sph(rng.uniform(0, 1.45), rng.uniform(0, 2 * math.pi)))
        m = W.material_cook_torrance(kd, alpha, n_idx, 0.1)
        D, F, G, f = orc.ct_terms(m, n, l, v)
        # float32 material fields
        kd32, a32, n32 = (float(np.float32(x)) for x in (kd, alpha, n_idx))
        assert f == pytest.approx(reference_f(kd32, a32, n32, n, l, v), rel=1e-9)
        assert F == pytest.approx(fresnel_sine_tangent(n32, v @ unit(l + v)), rel=1e-9)
        assert 0 < G <= 1
        # reciprocity
        assert orc.ct_terms(m, n, v, l)[3] == pytest.approx(f, rel=1e-12)
    # below the horizon nothing is reflected
    m = W.material_cook_torrance(0.5, 0.5, 2.0, 0.0)
    assert orc.ct_terms(m, n, unit([0.3, 0, -0.2]), unit([0, 0, 1]))[3] == 0.0


def test_masking_limits(orc):
    n = (0.0, 0.0, 1.0)
    up = (0.0, 0.0, 1.0)
    for alpha in (0.05, 0.5, 1.0):
        assert orc.ct_terms(W.material_cook_torrance(0, alpha, 2, 0), n, up, up)[2] == pytest.approx(1.0, abs=1e-15)
    l = unit([1.0, 0.0, 0.3])
    assert orc.ct_terms(W.material_cook_torrance(0, 1e-4, 2, 0), n, l, l)[2] == pytest.approx(1.0, abs=1e-6)


@pytest.mark.parametrize("kd,alpha", [(1.0, 0.5), (0.0, 0.2), (0.0, 0.7), (0.3, 0.5)])
def test_energy_bound(orc, kd, alpha):
    """Directional albedo: exactly one for the diffuse part, at most one with
    the masked specular part."""
    m = W.material_cook_torrance(kd, alpha, 100.0, 0.0)
    n = (0.0, 0.0, 1.0)
    for tl in (0.0, 0.6, 1.2):
        l = sph(tl, 0.0)

        def integrand(phi, th):
            return orc.ct_terms(m, n, l, sph(th, phi))[3] * math.cos(th) * math.sin(th)

        val, _ = integrate.dblquad(integrand, 0.0, math.pi / 2, 0.0, 2 * math.pi, epsabs=1e-6, epsrel=1e-5)
        if kd == 1.0:
            assert val == pytest.approx(1.0, abs=1e-5)
        else:
            assert 0.0 < val <= 1.0 + 1e-4


def test_diffuse_plane_closed_form(orc):
    """k_d = 1: f = 1/pi, so each primary returns E0 rho cos(theta) Omega / pi
    with Omega the solid angle of the beam window."""
    dr, dist, rho = 0.044, 100.5 * 0.044, 0.7
    m = W.material_cook_torrance(1.0, 0.5, 1.5, 1.0 - rho)
    s = W.plane_scene(dist, m, n_azimuth=1, rays_per_beam=256, max_bounces=1, n_bins=1024,
                      bin_size_m=dr, seed=77)
    out = orc.scan_scene(s)
    b = s.params["beam_width_rad"]
    omega = 2 * math.pi * (1 - math.cos(np.float32(b) / 2))
    E0 = float(np.float32(1.0) / np.float32(256))
    want = ret = 0.0
    for i in range(256):
        p = orc.primary(s.params, s.pose, 0, i)
        cos_t = float(p["d"][0])
        w = cos_t * omega / math.pi
        want += E0 * float(np.float32(rho)) * w * float(p["g"])
        ret += E0 * float(np.float32(rho)) * w
    img = out["image"][0]
    assert np.nonzero(img)[0].tolist() == [100]
    assert img[100] == pytest.approx(want, rel=1e-6)
    e = dict(zip(orc.E_SLOTS, out["energy"][0]))
    assert e["returned_in"] == pytest.approx(ret, rel=1e-6)
    assert e["absorbed"] == pytest.approx(0.0, abs=1e-15)


def test_transmitted_share_refracts(orc):
    """A Cook-Torrance slab passes 1 - rho of the energy into the material,
    where it continues by Snell's law (records show the refracted child)."""
    m = W.material_cook_torrance(0.2, 0.5, 2.0, 0.25)
    s = W.slab_scene(2.0, 0.05, m, n_azimuth=1, rays_per_beam=16, max_bounces=2, n_bins=256, bin_size_m=0.044)
    out = orc.scan_scene(s, records=True)
    rec = out["records"]
    assert (rec[:, 0] >= 0).all() and (rec[:, 2] >= 0).all()  # refracted child hits the back face
    e = dict(zip(orc.E_SLOTS, out["energy"].sum(axis=0)))
    assert sum(e[k] for k in orc.E_SLOTS[1:]) == pytest.approx(e["emitted"], rel=1e-12)


def test_elliptic_stretch_scales_the_cone(orc):
    base = W.sensor_params(1, 64, 1, 16)
    wide = dict(base, beam_stretch_az=2.0, beam_stretch_inc=0.5)
    pose = W.identity_pose()
    for i in range(64):
        a, b = orc.primary(base, pose, 0, i), orc.primary(wide, pose, 0, i)
        az_a, az_b = math.atan2(a["d"][1], a["d"][0]), math.atan2(b["d"][1], b["d"][0])
        inc_a, inc_b = math.asin(a["d"][2]), math.asin(b["d"][2])
        assert az_b == pytest.approx(2.0 * az_a, abs=2e-7)
        assert inc_b == pytest.approx(0.5 * inc_a, abs=2e-7)
        assert a["g"] == b["g"] and a["z"] == b["z"]
    same = orc.primary(dict(base, beam_stretch_az=1.0, beam_stretch_inc=1.0), pose, 0, 5)
    assert np.array_equal(same["d"], orc.primary(base, pose, 0, 5)["d"])
