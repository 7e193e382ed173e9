"""Seeded sensor trajectories and scan-request streams on the large scene,
and seeded poses inside the tiny room."""
from __future__ import annotations

import math

import numpy as np

from .scenes import BLOCK, PITCH, N_LOTS, ROOM_LO, ROOM_HI, sensor_params, yaw_pose


def street_points(rng, n: int, tiles: int = 3):
    """Random points on street centre lines (x or y a multiple of the street
    pitch), away from the block border, at sensor height 1.5 m."""
    span = tiles * BLOCK
    pts = []
    while len(pts) < n:
        along = rng.uniform(PITCH * 0.5, span - PITCH * 0.5)
        line = int(rng.integers(1, tiles * N_LOTS)) * PITCH
        if rng.integers(2):
            pts.append((line, along, 1.5))
        else:
            pts.append((along, line, 1.5))
    return np.array(pts, dtype=np.float64)


def _catmull_rom(P, n_samples: int):
    """Uniform Catmull-Rom spline through P (open, end points duplicated),
    resampled to n_samples points equally spaced in arc length."""
    P = np.asarray(P, dtype=np.float64)
    Q = np.concatenate([P[:1], P, P[-1:]])
    dense = []
    for i in range(1, len(Q) - 2):
        p0, p1, p2, p3 = Q[i - 1], Q[i], Q[i + 1], Q[i + 2]
        for t in np.linspace(0.0, 1.0, 200, endpoint=False):
            t2, t3 = t * t, t * t * t
            dense.append(0.5 * ((2 * p1) + (-p0 + p2) * t
                                + (2 * p0 - 5 * p1 + 4 * p2 - p3) * t2
                                + (-p0 + 3 * p1 - 3 * p2 + p3) * t3))
    dense.append(P[-1])
    dense = np.array(dense)
    seg = np.linalg.norm(np.diff(dense[:, :2], axis=0), axis=1)
    s = np.concatenate([[0.0], np.cumsum(seg)])
    targets = np.linspace(0.0, s[-1], n_samples)
    x = np.interp(targets, s, dense[:, 0])
    y = np.interp(targets, s, dense[:, 1])
    return np.column_stack([x, y]), s[-1]


def spline_poses(seed: int = 4, n_poses: int = 64, n_knots: int = 8,
                 max_bounces: int = 5, n_bins: int = 3776, **kw):
    """64 poses equally spaced in arc length on a Catmull-Rom spline through 8
    seeded street points of the large scene, z = 1.5 m, yaw along the tangent.
    Each scan draws rays/beam from {256, 1024, 4096} and azimuths from
    {100, 400, 800}.  Returns a list of (pose, params)."""
    rng = np.random.default_rng(seed)
    knots = street_points(rng, n_knots)
    xy, _ = _catmull_rom(knots[:, :2], n_poses)
    tang = np.gradient(xy, axis=0)
    out = []
    for i in range(n_poses):
        yaw = math.atan2(tang[i, 1], tang[i, 0])
        pose = yaw_pose((xy[i, 0], xy[i, 1], 1.5), yaw)
        params = sensor_params(int(rng.choice([100, 400, 800])),
                               int(rng.choice([256, 1024, 4096])),
                               max_bounces, n_bins, scan_id=i, **kw)
        out.append((pose, params))
    return out


def room_poses(room, seed: int = 6, n_poses: int = 64, n_azimuth: int = 400,
               rays_per_beam: int = 64, max_bounces: int = 3, n_bins: int = 1024, **kw):
    """``n_poses`` seeded poses inside the tiny room ``room`` (a Scene from
    ``tiny_room``): x, y uniform at least 0.5 m from the walls and 0.2 m clear
    of every cuboid's bounding circle, z = 0 (1 m above the floor), yaw
    uniform; every scan has the room's own sensor settings.  Returns a list
    of (pose, params)."""
    rng = np.random.default_rng(seed)
    circles = room.meta["cuboids"]
    out = []
    while len(out) < n_poses:
        x = rng.uniform(ROOM_LO[0] + 0.5, ROOM_HI[0] - 0.5)
        y = rng.uniform(ROOM_LO[1] + 0.5, ROOM_HI[1] - 0.5)
        yaw = rng.uniform(-math.pi, math.pi)
        if any(math.hypot(x - cx, y - cy) < r + 0.2 for cx, cy, r in circles):
            continue
        params = sensor_params(n_azimuth, rays_per_beam, max_bounces, n_bins,
                               scan_id=len(out), **kw)
        out.append((yaw_pose((x, y, 0.0), yaw), params))
    return out


def request_stream(seed: int = 5, rate_hz: float = 200.0, duration_s: float = 60.0,
                   n_robots: int = 32, n_bins: int = 3776, **kw):
    """Poisson stream of scan requests from ``n_robots`` robots on the large
    scene.  Each request: arrival time, robot id, a random street pose with a
    random yaw, azimuths ~ U{100..800}, rays/beam ~ U{256..4096},
    bounces ~ U{2..5}."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        p = street_points(rng, 1)[0]
        pose = yaw_pose(p, rng.uniform(-math.pi, math.pi))
        params = sensor_params(int(rng.integers(100, 801)), int(rng.integers(256, 4097)),
                               int(rng.integers(2, 6)), n_bins,
                               scan_id=len(reqs), **kw)
        reqs.append(dict(t_arrival=t, robot=int(rng.integers(n_robots)),
                         pose=pose, params=params))
    return reqs
