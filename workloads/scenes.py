"""Seeded synthetic scenes and scan parameters.

Every mesh is closed and wound so that the geometric normal
``(v1 - v0) x (v2 - v0)`` points out of the solid (room walls, which enclose
the sensor, point into the room).  Arrays are plain numpy:

* ``vertices``     float32 [nv, 3]  (metres)
* ``indices``      uint32  [nt, 3]
* ``tri_material`` uint16  [nt]     (index into ``materials``)

Materials follow the parameterisation of the paper's standard BRDF
(Sec. III-A, Eq. 5): ``A`` diffuse share, ``B`` first glossy share, ``C``
exponent of the second glossy share, ``S = 1 - A - B``.  Roughness ``rho``
maps to ``A = rho/2, B = 0, C = min(2000, 2/rho^2 - 2)`` (the Phong exponent
that matches a Beckmann lobe of width ``rho``, Walter et al. 2007); a smooth
surface gets the paper's hardest lobe ``C = 2000`` (Sec. IV-B material table).

Nothing here samples rays or evaluates the radar model.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FLAG_BEAM_GAIN = 1
FLAG_FIXED_PATTERN = 2
FLAG_MIRROR_PAIRS = 4
FLAG_RETURN_ALL = 8
FLAG_AIR_PATH = 16

KIND_DIELECTRIC = 0
KIND_METAL = 1
KIND_LAMBERTIAN = 2
KIND_COOK_TORRANCE = 3


# --------------------------------------------------------------------------
# materials, poses, parameters
# --------------------------------------------------------------------------
def material_metal(reflectance: float = 0.95, C: float = 2000.0) -> dict:
    return dict(kind=KIND_METAL, n=1.0, reflectance=float(reflectance),
                A=0.0, B=0.0, C=float(C))


def material_cook_torrance(diffuse: float, roughness: float, n: float, transmittance: float) -> dict:
    """Cook-Torrance microfacet material: diffuse amount k_d (A), GGX
    roughness (B), Fresnel index n, reflected share 1 - transmittance."""
    return dict(kind=KIND_COOK_TORRANCE, n=float(n), reflectance=float(1.0 - transmittance),
                A=float(diffuse), B=float(roughness), C=0.0)


def material_dielectric(n: float, roughness: float = 0.0) -> dict:
    rho = float(roughness)
    if rho <= 0.0:
        A, C = 0.0, 2000.0
    else:
        A, C = rho / 2.0, min(2000.0, 2.0 / (rho * rho) - 2.0)
    return dict(kind=KIND_DIELECTRIC, n=float(n), reflectance=0.0,
                A=A, B=0.0, C=C)


def material_lambertian(albedo: float) -> dict:
    return dict(kind=KIND_LAMBERTIAN, n=1.0, reflectance=float(albedo),
                A=1.0, B=0.0, C=1.0)


def identity_pose(position=(0.0, 0.0, 0.0)) -> dict:
    return dict(position=tuple(float(x) for x in position),
                quat_wxyz=(1.0, 0.0, 0.0, 0.0))


def yaw_pose(position, yaw: float) -> dict:
    return dict(position=tuple(float(x) for x in position),
                quat_wxyz=(math.cos(yaw / 2.0), 0.0, 0.0, math.sin(yaw / 2.0)))


def sensor_params(n_azimuth: int, rays_per_beam: int, max_bounces: int,
                  n_bins: int, bin_size_m: float = 0.044,
                  beam_width_deg: float = 2.0, beam_prob: float = 0.9,
                  energy_cutoff: float = 1e-12, seed: int = 0x5EED,
                  scan_id: int = 0, flags: int = FLAG_BEAM_GAIN,
                  beam_width_rad: float | None = None, beam_stretch_az: float = 0.0,
                  beam_stretch_inc: float = 0.0) -> dict:
    b = math.radians(beam_width_deg) if beam_width_rad is None else beam_width_rad
    return dict(n_azimuth=int(n_azimuth), rays_per_beam=int(rays_per_beam),
                max_bounces=int(max_bounces), n_bins=int(n_bins),
                bin_size_m=float(bin_size_m), beam_width_rad=float(b),
                beam_prob=float(beam_prob), energy_cutoff=float(energy_cutoff),
                seed=int(seed), scan_id=int(scan_id), flags=int(flags),
                beam_stretch_az=float(beam_stretch_az), beam_stretch_inc=float(beam_stretch_inc))


@dataclass
class Scene:
    name: str
    vertices: np.ndarray
    indices: np.ndarray
    tri_material: np.ndarray
    materials: list
    pose: dict
    params: dict
    meta: dict = field(default_factory=dict)

    @property
    def n_tris(self) -> int:
        return int(self.indices.shape[0])


# --------------------------------------------------------------------------
# mesh assembly
# --------------------------------------------------------------------------
class _Mesh:
    def __init__(self):
        self._v, self._f, self._m = [], [], []
        self._nv = 0

    def add(self, verts, tris, mat: int):
        verts = np.asarray(verts, dtype=np.float64).reshape(-1, 3)
        tris = np.asarray(tris, dtype=np.int64).reshape(-1, 3)
        self._v.append(verts)
        self._f.append(tris + self._nv)
        self._m.append(np.full(len(tris), mat, dtype=np.uint16))
        self._nv += len(verts)
        return len(tris)

    @property
    def n_tris(self) -> int:
        return int(sum(len(f) for f in self._f))

    def arrays(self):
        V = np.concatenate(self._v).astype(np.float32)
        F = np.concatenate(self._f).astype(np.uint32)
        M = np.concatenate(self._m).astype(np.uint16)
        return V, F, M


# corner index = ix + 2*iy + 4*iz ; quads listed counter-clockwise seen from
# outside the box
_BOX_QUADS = (
    (0, 2, 3, 1),  # -z
    (4, 5, 7, 6),  # +z
    (0, 1, 5, 4),  # -y
    (2, 6, 7, 3),  # +y
    (0, 4, 6, 2),  # -x
    (1, 3, 7, 5),  # +x
)


def _quads_to_tris(quads, flip=False):
    out = []
    for a, b, c, d in quads:
        if flip:
            out += [(a, c, b), (a, d, c)]
        else:
            out += [(a, b, c), (a, c, d)]
    return np.array(out, dtype=np.int64)


def box_mesh(lo, hi, yaw: float = 0.0, centre_xy=None, inward: bool = False):
    """Corners and 12 triangles of a box; optional yaw about the box centre."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    corners = np.array([[(hi if (c >> a) & 1 else lo)[a] for a in range(3)]
                        for c in range(8)], dtype=np.float64)
    if yaw != 0.0:
        cx, cy = ((lo[:2] + hi[:2]) / 2.0) if centre_xy is None else centre_xy
        c, s = math.cos(yaw), math.sin(yaw)
        x = corners[:, 0] - cx
        y = corners[:, 1] - cy
        corners[:, 0] = cx + c * x - s * y
        corners[:, 1] = cy + s * x + c * y
    return corners, _quads_to_tris(_BOX_QUADS, flip=inward)


def frame_box_mesh(origin, t, nrm, up, size_t, size_n, size_u):
    """Box spanned from ``origin`` by size_t*t, size_n*nrm, size_u*up with a
    right-handed frame (t, nrm, up)."""
    o = np.asarray(origin, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    nrm = np.asarray(nrm, dtype=np.float64)
    up = np.asarray(up, dtype=np.float64)
    corners = np.array([o + ((c & 1) * size_t) * t + (((c >> 1) & 1) * size_n) * nrm
                        + (((c >> 2) & 1) * size_u) * up for c in range(8)])
    # (t, nrm, up) right-handed => same winding as the axis box
    handed = float(np.dot(np.cross(t, nrm), up))
    return corners, _quads_to_tris(_BOX_QUADS, flip=handed < 0)


def prism_mesh(poly_xy, z0: float, z1: float):
    """Closed prism over a convex polygon given counter-clockwise from above."""
    p = np.asarray(poly_xy, dtype=np.float64)
    k = len(p)
    bot = np.column_stack([p, np.full(k, z0)])
    top = np.column_stack([p, np.full(k, z1)])
    verts = np.concatenate([bot, top])
    tris = []
    for i in range(k):
        j = (i + 1) % k
        tris += [(i, j, k + j), (i, k + j, k + i)]
    for i in range(1, k - 1):
        tris.append((k, k + i, k + i + 1))      # top, normal +z
        tris.append((0, i + 1, i))              # bottom, normal -z
    return verts, np.array(tris, dtype=np.int64)


def cone_mesh(cx, cy, z0, radius, height, segments=16):
    ang = 2.0 * math.pi * np.arange(segments) / segments
    base = np.column_stack([cx + radius * np.cos(ang), cy + radius * np.sin(ang),
                            np.full(segments, z0)])
    apex = np.array([[cx, cy, z0 + height]])
    verts = np.concatenate([base, apex])
    a = segments
    tris = [(i, (i + 1) % segments, a) for i in range(segments)]
    tris += [(0, i + 1, i) for i in range(1, segments - 1)]
    return verts, np.array(tris, dtype=np.int64)


def cylinder_mesh(cx, cy, z0, radius, height, segments=16):
    ang = 2.0 * math.pi * np.arange(segments) / segments
    poly = np.column_stack([cx + radius * np.cos(ang), cy + radius * np.sin(ang)])
    return prism_mesh(poly, z0, z0 + height)


def ground_grid(x0, y0, x1, y1, n, z=0.0):
    xs = np.linspace(x0, x1, n + 1)
    ys = np.linspace(y0, y1, n + 1)
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    verts = np.column_stack([X.ravel(), Y.ravel(), np.full(X.size, z)])
    tris = []
    w = n + 1
    for j in range(n):
        for i in range(n):
            a = j * w + i
            b, c, d = a + 1, a + w + 1, a + w
            tris += [(a, b, c), (a, c, d)]
    return verts, np.array(tris, dtype=np.int64)


def _finish(name, mesh: _Mesh, materials, pose, params, meta=None) -> Scene:
    V, F, M = mesh.arrays()
    return Scene(name, V, F, M, list(materials), pose, params, dict(meta or {}))


# --------------------------------------------------------------------------
# tiny room (10 x 8 x 3 m, four seeded cuboids)
# --------------------------------------------------------------------------
ROOM_LO = (-5.0, -4.0, -1.0)
ROOM_HI = (5.0, 4.0, 2.0)


def tiny_room(seed: int = 1, n_azimuth: int = 400, rays_per_beam: int = 64,
              max_bounces: int = 3, n_bins: int = 1024, **kw) -> Scene:
    """10x8x3 m Lambertian room around the sensor (1 m above the floor) with
    four seeded cuboids: 0 and 2 metal, 1 and 3 dielectric (n = 2.5)."""
    rng = np.random.default_rng(seed)
    mats = [material_lambertian(0.3), material_metal(0.95), material_dielectric(2.5)]
    mesh = _Mesh()
    v, f = box_mesh(ROOM_LO, ROOM_HI, inward=True)
    mesh.add(v, f, 0)
    placed = []
    while len(placed) < 4:
        cx, cy = rng.uniform(-4.0, 4.0), rng.uniform(-3.0, 3.0)
        wx, wy = rng.uniform(0.3, 1.5), rng.uniform(0.3, 1.5)
        h = rng.uniform(0.5, 2.5)
        yaw = rng.uniform(0.0, math.pi / 2.0)
        r = 0.5 * math.hypot(wx, wy)
        if math.hypot(cx, cy) < 1.0 + r:
            continue
        if abs(cx) + r > 4.9 or abs(cy) + r > 3.9:
            continue
        if any(math.hypot(cx - px, cy - py) < r + pr + 0.05 for px, py, pr in placed):
            continue
        placed.append((cx, cy, r))
        v, f = box_mesh((cx - wx / 2, cy - wy / 2, ROOM_LO[2]),
                        (cx + wx / 2, cy + wy / 2, ROOM_LO[2] + h), yaw=yaw)
        mesh.add(v, f, 1 if len(placed) in (1, 3) else 2)
    params = sensor_params(n_azimuth, rays_per_beam, max_bounces, n_bins, **kw)
    return _finish("tiny_room", mesh, mats, identity_pose(), params,
                   dict(seed=seed, cuboids=placed))


def empty_room(albedo: float = 0.3, **kw) -> Scene:
    mesh = _Mesh()
    v, f = box_mesh(ROOM_LO, ROOM_HI, inward=True)
    mesh.add(v, f, 0)
    params = sensor_params(kw.pop("n_azimuth", 400), kw.pop("rays_per_beam", 16),
                           kw.pop("max_bounces", 1), kw.pop("n_bins", 1024), **kw)
    return _finish("empty_room", mesh, [material_lambertian(albedo)],
                   identity_pose(), params)


def plane_scene(distance: float, material: dict, half_size: float = 20.0,
                **kw) -> Scene:
    """A single square (2 triangles) at x = distance facing the sensor."""
    d, s = float(distance), float(half_size)
    verts = [(d, -s, -s), (d, s, -s), (d, s, s), (d, -s, s)]
    # normal must point to -x (towards the sensor): (v1-v0) x (v2-v0)
    tris = [(0, 2, 1), (0, 3, 2)]
    mesh = _Mesh()
    mesh.add(verts, tris, 0)
    params = sensor_params(kw.pop("n_azimuth", 1), kw.pop("rays_per_beam", 256),
                           kw.pop("max_bounces", 1), kw.pop("n_bins", 1024), **kw)
    return _finish("plane", mesh, [material], identity_pose(), params)


def slab_scene(distance: float, thickness: float, material: dict,
               half_size: float = 20.0, **kw) -> Scene:
    """Closed slab x in [d, d + h], large in y and z."""
    d, h, s = float(distance), float(thickness), float(half_size)
    mesh = _Mesh()
    v, f = box_mesh((d, -s, -s), (d + h, s, s))
    mesh.add(v, f, 0)
    params = sensor_params(kw.pop("n_azimuth", 1), kw.pop("rays_per_beam", 256),
                           kw.pop("max_bounces", 2), kw.pop("n_bins", 1024), **kw)
    return _finish("slab", mesh, [material], identity_pose(), params)


def single_triangle_scene(v0, v1, v2, material: dict, **kw) -> Scene:
    mesh = _Mesh()
    mesh.add([v0, v1, v2], [(0, 1, 2)], 0)
    params = sensor_params(kw.pop("n_azimuth", 8), kw.pop("rays_per_beam", 8),
                           kw.pop("max_bounces", 2), kw.pop("n_bins", 256), **kw)
    return _finish("triangle", mesh, [material], identity_pose(), params)


def mirror_scene(seed: int = 7, **kw) -> Scene:
    """Room with cuboids placed in mirror pairs about the plane y = 0."""
    rng = np.random.default_rng(seed)
    mats = [material_lambertian(0.3), material_metal(0.95), material_dielectric(2.5)]
    mesh = _Mesh()
    v, f = box_mesh(ROOM_LO, ROOM_HI, inward=True)
    mesh.add(v, f, 0)
    for i in range(3):
        cx = rng.uniform(-3.5, 3.5)
        cy = rng.uniform(1.4, 2.6)
        wx, wy = rng.uniform(0.3, 1.0), rng.uniform(0.3, 1.0)
        h = rng.uniform(0.5, 2.5)
        mat = 1 + (i % 2)
        for sgn in (1.0, -1.0):
            y0, y1 = sorted((sgn * (cy - wy / 2), sgn * (cy + wy / 2)))
            v, f = box_mesh((cx - wx / 2, y0, ROOM_LO[2]), (cx + wx / 2, y1, ROOM_LO[2] + h))
            mesh.add(v, f, mat)
    params = sensor_params(kw.pop("n_azimuth", 64), kw.pop("rays_per_beam", 32),
                           kw.pop("max_bounces", 3), kw.pop("n_bins", 1024), **kw)
    return _finish("mirror_room", mesh, mats, identity_pose(), params)


def thin_pillars_scene(seed: int = 11, **kw) -> Scene:
    """Thin metal pillars inside a hall whose walls are a nearly transparent
    dielectric (n = 1.05), after the wheel-loader hall of Sec. IV-F."""
    rng = np.random.default_rng(seed)
    mats = [material_dielectric(1.05), material_metal(0.95)]
    mesh = _Mesh()
    v, f = box_mesh((-12.0, -9.0, -1.0), (12.0, 9.0, 6.0))
    mesh.add(v, f, 0)  # hall walls, wound outward: the sensor is inside the medium boundary
    for _ in range(10):
        cx, cy = rng.uniform(-10, 10), rng.uniform(-7, 7)
        if math.hypot(cx, cy) < 2.0:
            continue
        v, f = cylinder_mesh(cx, cy, -1.0, 0.12, 6.5, segments=12)
        mesh.add(v, f, 1)
    params = sensor_params(kw.pop("n_azimuth", 100), kw.pop("rays_per_beam", 64),
                           kw.pop("max_bounces", 2), kw.pop("n_bins", 1024), **kw)
    return _finish("thin_pillars", mesh, mats, identity_pose(), params)


def transform_scene(scene: Scene, yaw: float = 0.0, shift=(0.0, 0.0, 0.0)) -> Scene:
    """Rotate the mesh about +z by ``yaw`` and then translate it (float64 maths,
    rounded to float32); the pose position is moved the same way."""
    c, s = math.cos(yaw), math.sin(yaw)
    V = scene.vertices.astype(np.float64)
    x, y = V[:, 0].copy(), V[:, 1].copy()
    V[:, 0] = c * x - s * y + shift[0]
    V[:, 1] = s * x + c * y + shift[1]
    V[:, 2] = V[:, 2] + shift[2]
    p = np.asarray(scene.pose["position"], dtype=np.float64)
    p2 = (c * p[0] - s * p[1] + shift[0], s * p[0] + c * p[1] + shift[1], p[2] + shift[2])
    pose = dict(position=tuple(float(np.float32(q)) for q in p2),
                quat_wxyz=scene.pose["quat_wxyz"])
    return Scene(scene.name + "_xf", V.astype(np.float32), scene.indices.copy(),
                 scene.tri_material.copy(), list(scene.materials), pose,
                 dict(scene.params), dict(scene.meta))


# --------------------------------------------------------------------------
# procedural urban block (about 200k triangles)
# --------------------------------------------------------------------------
BLOCK = 256.0
PITCH = 32.0          # street pitch: 24 m lots + 8 m streets
STREET_HALF = 4.0
N_LOTS = 8


def _convex_footprint(rng, cx, cy, radius):
    k = int(rng.integers(4, 13))
    ang = np.sort(rng.uniform(0.0, 2.0 * math.pi, size=k))
    # keep the polygon fat: no angular gap above 120 degrees
    while np.max(np.diff(np.concatenate([ang, [ang[0] + 2 * math.pi]]))) > 2.1:
        ang = np.sort(rng.uniform(0.0, 2.0 * math.pi, size=k))
    sx, sy = rng.uniform(0.75, 1.0), rng.uniform(0.75, 1.0)
    rot = rng.uniform(0.0, math.pi)
    x = radius * sx * np.cos(ang)
    y = radius * sy * np.sin(ang)
    c, s = math.cos(rot), math.sin(rot)
    return np.column_stack([cx + c * x - s * y, cy + s * x + c * y])


def _urban_objects(rng, n_materials=12):
    """Returns a list of (verts, tris, material, kind, extra) objects."""
    objs = []
    # buildings: 2..4 per lot inside a 19 x 19 m inner region
    for li in range(N_LOTS):
        for lj in range(N_LOTS):
            x0 = li * PITCH + STREET_HALF + 2.5
            y0 = lj * PITCH + STREET_HALF + 2.5
            inner = PITCH - 2 * STREET_HALF - 5.0
            want = int(rng.integers(3, 6))
            placed = []
            tries = 0
            while len(placed) < want and tries < 200:
                tries += 1
                r = rng.uniform(2.5, 5.0)
                cx = rng.uniform(x0 + r, x0 + inner - r)
                cy = rng.uniform(y0 + r, y0 + inner - r)
                if any(math.hypot(cx - px, cy - py) < r + pr + 0.5 for px, py, pr in placed):
                    continue
                placed.append((cx, cy, r))
                poly = _convex_footprint(rng, cx, cy, r)
                h = rng.uniform(6.0, 40.0)
                v, f = prism_mesh(poly, 0.0, h)
                objs.append((v, f, int(rng.integers(n_materials)), "building",
                             dict(poly=poly, height=h)))
    # cars: two stacked boxes, in two lanes of every street, both directions
    for axis in (0, 1):
        for si in range(N_LOTS + 1):
            for lane in (-2.0, 2.0):
                c_line = si * PITCH + lane
                if c_line < 1.0 or c_line > BLOCK - 1.0:
                    continue
                pos = rng.uniform(0.0, 4.0)
                while pos < BLOCK - 4.5:
                    L, W = rng.uniform(3.8, 4.6), rng.uniform(1.6, 1.9)
                    mat = int(rng.integers(n_materials))
                    if axis == 0:   # street runs along y at x = c_line
                        lo1, hi1 = (c_line - W / 2, pos, 0.25), (c_line + W / 2, pos + L, 1.0)
                        lo2, hi2 = (c_line - W / 2 + 0.1, pos + 0.9, 1.0), (c_line + W / 2 - 0.1, pos + L - 1.1, 1.5)
                    else:
                        lo1, hi1 = (pos, c_line - W / 2, 0.25), (pos + L, c_line + W / 2, 1.0)
                        lo2, hi2 = (pos + 0.9, c_line - W / 2 + 0.1, 1.0), (pos + L - 1.1, c_line + W / 2 - 0.1, 1.5)
                    v1, f1 = box_mesh(lo1, hi1)
                    v2, f2 = box_mesh(lo2, hi2)
                    objs.append((np.concatenate([v1, v2]), np.concatenate([f1, f2 + 8]),
                                 mat, "car", {}))
                    pos += L + rng.uniform(0.5, 1.6)
    # trees on the sidewalk ring of every lot
    for li in range(N_LOTS):
        for lj in range(N_LOTS):
            x0 = li * PITCH + STREET_HALF + 1.2
            y0 = lj * PITCH + STREET_HALF + 1.2
            side = PITCH - 2 * STREET_HALF - 2.4
            for e in range(4):
                pos = rng.uniform(0.0, 2.0)
                while pos < side:
                    if e == 0:
                        cx, cy = x0 + pos, y0
                    elif e == 1:
                        cx, cy = x0 + side, y0 + pos
                    elif e == 2:
                        cx, cy = x0 + side - pos, y0 + side
                    else:
                        cx, cy = x0, y0 + side - pos
                    th = rng.uniform(1.5, 3.0)
                    v1, f1 = cylinder_mesh(cx, cy, 0.0, rng.uniform(0.12, 0.25), th)
                    v2, f2 = cone_mesh(cx, cy, th, rng.uniform(0.8, 1.6), rng.uniform(2.5, 6.0))
                    objs.append((np.concatenate([v1, v2]), np.concatenate([f1, f2 + len(v1)]),
                                 int(rng.integers(n_materials)), "tree", {}))
                    pos += rng.uniform(2.5, 4.5)
    return objs


def _urban_mesh(seed: int, target: int = 200_000, n_materials: int = 12):
    rng = np.random.default_rng(seed)
    mats = [material_dielectric(rng.uniform(1.5, 6.0), rng.uniform(0.0, 0.5))
            for _ in range(n_materials)]
    objs = _urban_objects(rng, n_materials)
    n_obj_tris = sum(len(o[1]) for o in objs)
    g = max(1, int(round(math.sqrt(max(target - n_obj_tris, 2) / 2.0))))
    mesh = _Mesh()
    v, f = ground_grid(0.0, 0.0, BLOCK, BLOCK, g)
    mesh.add(v, f, int(rng.integers(n_materials)))
    for v, f, m, _, _ in objs:
        mesh.add(v, f, m)
    buildings = [o[4] for o in objs if o[3] == "building"]
    counts = dict(ground=2 * g * g,
                  building=sum(len(o[1]) for o in objs if o[3] == "building"),
                  car=sum(len(o[1]) for o in objs if o[3] == "car"),
                  tree=sum(len(o[1]) for o in objs if o[3] == "tree"))
    return mesh, mats, buildings, counts


URBAN_SENSOR = (4 * PITCH, 4.5 * PITCH, 1.5)


def urban_block(seed: int = 2, n_azimuth: int = 400, rays_per_beam: int = 1024,
                max_bounces: int = 4, n_bins: int = 3776, **kw) -> Scene:
    """256 x 256 m block: ground grid, extruded convex buildings, two-box cars,
    cylinder+cone trees; 12 dielectric materials n~U[1.5,6], roughness~U[0,0.5]."""
    mesh, mats, buildings, counts = _urban_mesh(seed)
    params = sensor_params(n_azimuth, rays_per_beam, max_bounces, n_bins, **kw)
    return _finish("urban_block", mesh, mats, identity_pose(URBAN_SENSOR), params,
                   dict(seed=seed, counts=counts, n_tris=mesh.n_tris))


# --------------------------------------------------------------------------
# large scene: urban block tiled 3 x 3 + 1 cm glass panels on facades
# --------------------------------------------------------------------------
def _facade_slots(buildings):
    slots = []
    for b in buildings:
        poly, h = b["poly"], b["height"]
        k = len(poly)
        for i in range(k):
            p, q = poly[i], poly[(i + 1) % k]
            edge = q - p
            L = float(np.hypot(*edge))
            if L < 2.4:
                continue
            t = edge / L
            nrm = np.array([t[1], -t[0]])   # outward for a counter-clockwise polygon
            ncol = int((L - 0.4) // 2.5)
            nrow = int((h - 1.0) // 3.0)
            for c in range(ncol):
                for r in range(nrow):
                    slots.append((p, t, nrm, 0.2 + 2.5 * c, 1.0 + 3.0 * r))
    return slots


def large_scene(seed: int = 3, n_azimuth: int = 400, rays_per_beam: int = 4096,
                max_bounces: int = 5, n_bins: int = 3776,
                target: int = 2_000_000, **kw) -> Scene:
    """The urban block (seed 2) tiled 3x3, plus enough 1 cm thick glass panels
    (n = 2.0, smooth) on facades to reach about ``target`` triangles."""
    base_mesh, mats, buildings, counts = _urban_mesh(2)
    V0, F0, M0 = base_mesh.arrays()
    rng = np.random.default_rng(seed)
    glass = len(mats)
    mats = mats + [material_dielectric(2.0, 0.0)]
    Vs, Fs, Ms = [], [], []
    nv = 0
    for ti in range(3):
        for tj in range(3):
            Vs.append(V0.astype(np.float64) + np.array([ti * BLOCK, tj * BLOCK, 0.0]))
            Fs.append(F0.astype(np.int64) + nv)
            Ms.append(M0)
            nv += len(V0)
    n_panels = (target - 9 * len(F0)) // 12
    slots = _facade_slots(buildings)
    tiles = [(ti, tj) for ti in range(3) for tj in range(3)]
    all_slots = len(slots) * 9
    pick = rng.choice(all_slots, size=min(n_panels, all_slots), replace=False)
    up = np.array([0.0, 0.0, 1.0])
    pv, pf = [], []
    for idx in np.sort(pick):
        ti, tj = tiles[idx // len(slots)]
        p, t, nrm, off_t, off_z = slots[idx % len(slots)]
        w = rng.uniform(1.0, 2.0)
        base = np.array([p[0] + ti * BLOCK, p[1] + tj * BLOCK, off_z])
        base[:2] += t * off_t + nrm * 0.05
        t3 = np.array([t[0], t[1], 0.0])
        n3 = np.array([nrm[0], nrm[1], 0.0])
        v, f = frame_box_mesh(base, t3, n3, up, w, 0.01, 1.5)
        pv.append(v)
        pf.append(f + nv)
        nv += 8
    V = np.concatenate(Vs + pv).astype(np.float32)
    F = np.concatenate(Fs + pf).astype(np.uint32)
    M = np.concatenate(Ms + [np.full(12 * len(pv), glass, dtype=np.uint16)]).astype(np.uint16)
    sensor = (BLOCK + URBAN_SENSOR[0], BLOCK + URBAN_SENSOR[1], URBAN_SENSOR[2])
    params = sensor_params(n_azimuth, rays_per_beam, max_bounces, n_bins, **kw)
    meta = dict(seed=seed, base_counts=counts, n_base=int(len(F0)),
                n_panels=len(pv), n_tris=int(len(F)))
    return Scene("large_scene", V, F, M, mats, identity_pose(sensor), params, meta)
