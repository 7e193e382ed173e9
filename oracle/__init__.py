"""CPU oracle for the radar scan -- TEST INFRASTRUCTURE ONLY.

A ctypes wrapper around ``radar_oracle.c``: a plain brute-force tracer written
from the RadaRays paper (Sec. III) that tests every triangle for every ray
segment.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
may import this package; the HIP library never does, and this package never
imports the library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "radar_oracle.c")
_LIB = os.environ.get("RADAR_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

CFLAGS = ["-O2", "-std=gnu11", "-fPIC", "-shared", "-pthread", "-ffp-contract=off",
          "-fno-fast-math", "-fexcess-precision=standard"]

E_SLOTS = ("emitted", "returned_in", "returned_out", "escaped", "absorbed",
           "terminated", "cut", "blocked")
FLAG_AIR_PATH = 16


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Pose(C.Structure):
    _fields_ = [("position", C.c_float * 3), ("quat_wxyz", C.c_float * 4)]


class Params(C.Structure):
    _fields_ = [("n_azimuth", C.c_uint32), ("rays_per_beam", C.c_uint32),
                ("max_bounces", C.c_uint32), ("n_bins", C.c_uint32),
                ("bin_size_m", C.c_float), ("beam_width_rad", C.c_float),
                ("beam_prob", C.c_float), ("energy_cutoff", C.c_float),
                ("seed", C.c_uint64), ("scan_id", C.c_uint32), ("flags", C.c_uint32),
                ("stretch_az", C.c_float), ("stretch_inc", C.c_float)]


class PostParams(C.Structure):
    _fields_ = [("blur_sigma_bins", C.c_float), ("uniform_amp", C.c_float), ("perlin_amp", C.c_float),
                ("perlin_cell_az", C.c_float), ("perlin_cell_bins", C.c_float), ("db_floor", C.c_float),
                ("max_value", C.c_uint32), ("reserved0", C.c_uint32), ("seed", C.c_uint64),
                ("scan_id", C.c_uint32), ("reserved1", C.c_uint32)]


class Material(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("n", C.c_float), ("reflectance", C.c_float),
                ("A", C.c_float), ("B", C.c_float), ("C", C.c_float)]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            lib = C.CDLL(_LIB)
            P = C.POINTER
            lib.orc_philox4x64_10.argtypes = [P(C.c_uint64), P(C.c_uint64), P(C.c_uint64)]
            lib.orc_erfinv.restype = C.c_double
            lib.orc_erfinv.argtypes = [C.c_double]
            lib.orc_sigma_r.restype = C.c_double
            lib.orc_sigma_r.argtypes = [C.c_double, C.c_double]
            lib.orc_lobe_integral.restype = C.c_double
            lib.orc_lobe_integral.argtypes = [C.c_double]
            lib.orc_window_coeffs.argtypes = [P(Material), C.c_double, P(C.c_double)]
            lib.orc_ray_triangle.restype = C.c_int
            lib.orc_ray_triangle.argtypes = [P(C.c_float)] * 5 + [C.c_float, P(C.c_float)]
            lib.orc_offset.argtypes = [P(C.c_float), P(C.c_float), P(C.c_float)]
            lib.orc_primary.argtypes = [P(Params), P(Pose), C.c_uint32, C.c_uint32,
                                        P(C.c_float), P(C.c_float), P(C.c_float),
                                        P(C.c_double), P(C.c_double)]
            lib.orc_interact.argtypes = [P(C.c_float), P(C.c_float), P(Material), C.c_float,
                                         C.c_float, C.c_uint32, P(C.c_float), P(C.c_double)]
            lib.orc_scan.restype = C.c_int
            lib.orc_scan.argtypes = [P(C.c_float), C.c_uint32, P(C.c_uint32), C.c_uint32,
                                     P(C.c_uint16), P(Pose), P(Params), P(Material), C.c_uint32,
                                     P(C.c_uint32), C.c_uint32, P(C.c_uint8), P(C.c_double),
                                     P(C.c_int32), P(C.c_uint8), P(C.c_double),
                                     P(C.c_uint64), C.c_int]
            lib.orc_ct_terms.argtypes = [P(Material), P(C.c_double), P(C.c_double), P(C.c_double),
                                         P(C.c_double)]
            lib.orc_perlin.restype = C.c_double
            lib.orc_perlin.argtypes = [C.c_uint64, C.c_uint32, C.c_double, C.c_double]
            lib.orc_post.argtypes = [P(C.c_float), C.c_uint32, C.c_uint32, P(PostParams),
                                     P(C.c_float), P(C.c_uint8), P(C.c_double)]
            _lib = lib
    return _lib


def _f3(v):
    return (C.c_float * 3)(*[float(x) for x in v])


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


def make_pose(pose: dict) -> Pose:
    return Pose((C.c_float * 3)(*pose["position"]), (C.c_float * 4)(*pose["quat_wxyz"]))


def make_params(p: dict) -> Params:
    return Params(p["n_azimuth"], p["rays_per_beam"], p["max_bounces"], p["n_bins"],
                  p["bin_size_m"], p["beam_width_rad"], p["beam_prob"], p["energy_cutoff"],
                  p["seed"], p["scan_id"], p["flags"], p.get("beam_stretch_az", 0.0),
                  p.get("beam_stretch_inc", 0.0))


def make_material(m: dict) -> Material:
    return Material(m["kind"], m["n"], m["reflectance"], m["A"], m["B"], m["C"])


# ---------------------------------------------------------------- primitives
def philox4x64_10(key, ctr):
    lib = _load()
    k = (C.c_uint64 * 2)(*[int(x) for x in key])
    c = (C.c_uint64 * 4)(*[int(x) for x in ctr])
    out = (C.c_uint64 * 4)()
    lib.orc_philox4x64_10(k, c, out)
    return [int(x) for x in out]


def erfinv(p: float) -> float:
    return _load().orc_erfinv(p)


def sigma_r(beam_width: float, beam_prob: float) -> float:
    return _load().orc_sigma_r(beam_width, beam_prob)


def lobe_integral(Cexp: float) -> float:
    return _load().orc_lobe_integral(Cexp)


def window_coeffs(material: dict, beam_width: float):
    out = (C.c_double * 4)()
    m = make_material(material)
    _load().orc_window_coeffs(C.byref(m), beam_width, out)
    return dict(Z=out[0], a=out[1], beta=out[2], s=out[3])


def ray_triangle(o, d, v0, v1, v2, tmax=np.inf):
    t = C.c_float()
    hit = _load().orc_ray_triangle(_f3(o), _f3(d), _f3(v0), _f3(v1), _f3(v2),
                                   np.float32(tmax), C.byref(t))
    return float(t.value) if hit else None


def offset(p, n):
    out = (C.c_float * 3)()
    _load().orc_offset(_f3(p), _f3(n), out)
    return np.array(out[:], dtype=np.float32)


def primary(params: dict, pose: dict, k: int, i: int):
    o, d, g = (C.c_float * 3)(), (C.c_float * 3)(), C.c_float()
    z, om = C.c_double(), C.c_double()
    prm, ps = make_params(params), make_pose(pose)
    _load().orc_primary(C.byref(prm), C.byref(ps), k, i, o, d, C.byref(g), C.byref(z),
                        C.byref(om))
    return dict(o=np.array(o[:], np.float32), d=np.array(d[:], np.float32),
                g=np.float32(g.value), z=z.value, omega=om.value)


def interact(d, ng, material: dict, beam_width: float, n_cur: float = 1.0, flags: int = 0):
    of = (C.c_float * 12)()
    od = (C.c_double * 3)()
    m = make_material(material)
    _load().orc_interact(_f3(d), _f3(ng), C.byref(m), np.float32(beam_width),
                         np.float32(n_cur), flags, of, od)
    f = np.array(of[:], dtype=np.float32)
    return dict(entering=bool(f[0]), tir=bool(f[1]), has_refract=bool(f[2]),
                cosi=f[3], kappa=f[4], n2=f[5], refl=f[6:9], refr=f[9:12],
                R=od[0], T=od[1], w=od[2])


# ---------------------------------------------------------------- the scan
def scan(vertices, indices, tri_material, pose: dict, params: dict, materials,
         columns=None, primary_mask=None, records=False, exempt=False, energy=True,
         threads: int = 0):
    """Brute-force scan of the listed azimuth columns (all if None).

    Returns a dict with ``image`` float64 [n_cols, n_bins], ``columns``,
    ``segments`` (uint64 per column) and, if asked, ``records`` int32
    [n_cols * N_s, 2^B - 1], ``exempt`` bool [n_cols * N_s] and ``energy``
    float64 [n_cols, 8] (slots in E_SLOTS).  With the air-path flag,
    ``air_records`` int32 [n_cols * N_s, 2^B - 1] holds each hit's air-path
    outcome (-2 none, 0 returned, 1 blocked, 2 beyond the last bin).
    """
    lib = _load()
    V = np.ascontiguousarray(vertices, dtype=np.float32)
    F = np.ascontiguousarray(indices, dtype=np.uint32)
    M = np.ascontiguousarray(tri_material, dtype=np.uint16)
    prm = make_params(params)
    ps = make_pose(pose)
    mats = (Material * max(1, len(materials)))(*[make_material(m) for m in materials])
    if columns is None:
        cols = np.arange(params["n_azimuth"], dtype=np.uint32)
    else:
        cols = np.ascontiguousarray(columns, dtype=np.uint32)
    ncol = len(cols)
    nb, ns = params["n_bins"], params["rays_per_beam"]
    nheap = (1 << params["max_bounces"]) - 1
    img = np.zeros((ncol, nb), dtype=np.float64)
    air = bool(params.get("flags", 0) & FLAG_AIR_PATH)
    rec = np.empty((ncol * ns, 2 * nheap if air else nheap), dtype=np.int32) if records else None
    ex = np.zeros(ncol * ns, dtype=np.uint8) if exempt else None
    en = np.zeros((ncol, len(E_SLOTS)), dtype=np.float64) if energy else None
    segs = np.zeros(ncol, dtype=np.uint64)
    mask = None
    if primary_mask is not None:
        mask = np.ascontiguousarray(primary_mask, dtype=np.uint8)
        assert mask.size == params["n_azimuth"] * ns
    rc = lib.orc_scan(_ptr(V, C.c_float), V.shape[0], _ptr(F, C.c_uint32), F.shape[0],
                      _ptr(M, C.c_uint16), C.byref(ps), C.byref(prm), mats, len(materials),
                      _ptr(cols, C.c_uint32), ncol, _ptr(mask, C.c_uint8), _ptr(img, C.c_double),
                      _ptr(rec, C.c_int32), _ptr(ex, C.c_uint8), _ptr(en, C.c_double),
                      _ptr(segs, C.c_uint64), int(threads))
    if rc != 0:
        raise ValueError("oracle scan rejected its arguments")
    out = dict(image=img, columns=cols, segments=segs)
    if records:
        out["records"] = rec[:, :nheap]
        if air:
            out["air_records"] = rec[:, nheap:]
    if exempt:
        out["exempt"] = ex.astype(bool)
    if energy:
        out["energy"] = en
    return out


def scan_scene(scene, **kw):
    """``scan`` on a workloads.Scene (its own pose and params unless given)."""
    pose = kw.pop("pose", scene.pose)
    params = kw.pop("params", scene.params)
    return scan(scene.vertices, scene.indices, scene.tri_material, pose, params,
                scene.materials, **kw)


# ---------------------------------------------------------------- epilogue
POST_DEFAULTS = dict(blur_sigma_bins=0.0, uniform_amp=0.0, perlin_amp=0.0, perlin_cell_az=16.0,
                     perlin_cell_bins=64.0, db_floor=-100.0, max_value=255, seed=0x5EED, scan_id=0)


def make_post(p: dict) -> PostParams:
    q = dict(POST_DEFAULTS, **p)
    return PostParams(q["blur_sigma_bins"], q["uniform_amp"], q["perlin_amp"], q["perlin_cell_az"],
                      q["perlin_cell_bins"], q["db_floor"], q["max_value"], 0, q["seed"], q["scan_id"], 0)


def perlin(seed: int, scan_id: int, x: float, y: float) -> float:
    return float(_load().orc_perlin(seed, scan_id, x, y))


def postprocess(image, post: dict):
    """Blur, noise, dB and 8-bit map of a float32 [n_az][n_bins] image.
    Returns (dB float32, pixels uint8, pixel value before rounding float64)."""
    img = np.ascontiguousarray(image, dtype=np.float32)
    n_az, n_bins = img.shape
    db = np.empty_like(img)
    u8 = np.empty(img.shape, np.uint8)
    pre = np.empty(img.shape, np.float64)
    pp = make_post(post)
    _load().orc_post(_ptr(img, C.c_float), n_az, n_bins, C.byref(pp), _ptr(db, C.c_float),
                     _ptr(u8, C.c_uint8), _ptr(pre, C.c_double))
    return db, u8, pre


def ct_terms(material: dict, n, l, v):
    """Cook-Torrance terms (D, F, G1(n.l) G1(n.v), f) for unit vectors."""
    m = make_material(material)
    a = [(C.c_double * 3)(*[float(x) for x in vec]) for vec in (n, l, v)]
    out = (C.c_double * 4)()
    _load().orc_ct_terms(C.byref(m), a[0], a[1], a[2], out)
    return tuple(out[:])
