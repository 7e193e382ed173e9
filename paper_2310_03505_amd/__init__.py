"""Python binding of libradarays_hip.so, the MI355X radar-scan library.

Argument marshalling only: every step of a scan runs in the HIP library.
The functions keep the names of the C ABI (``include/radarays_hip.h``);
PyTorch provides device memory and the current stream.  The library must
have been built (``python -m paper_2310_03505_amd.build``); importing the
binding without it raises.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libradarays_hip.so")

RR_OK, RR_EINVAL, RR_ENOMEM, RR_EDEVICE, RR_ESTATE, RR_EOVERFLOW = 0, -1, -2, -3, -4, -5
RR_BEAM_GAIN, RR_FIXED_PATTERN, RR_MIRROR_PAIRS, RR_RETURN_ALL, RR_AIR_PATH = 1, 2, 4, 8, 16
RR_DIELECTRIC, RR_METAL, RR_LAMBERTIAN, RR_COOK_TORRANCE = 0, 1, 2, 3
RR_MAX_BOUNCES = 8


class RadarError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class rr_pose(C.Structure):
    _fields_ = [("position", C.c_float * 3), ("quat_wxyz", C.c_float * 4)]


class rr_sensor_params(C.Structure):
    _fields_ = [("n_azimuth", C.c_uint32), ("rays_per_beam", C.c_uint32),
                ("max_bounces", C.c_uint32), ("n_bins", C.c_uint32),
                ("bin_size_m", C.c_float), ("beam_width_rad", C.c_float),
                ("beam_prob", C.c_float), ("energy_cutoff", C.c_float),
                ("seed", C.c_uint64), ("scan_id", C.c_uint32), ("flags", C.c_uint32),
                ("beam_stretch_az", C.c_float), ("beam_stretch_inc", C.c_float)]


class rr_material(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("n", C.c_float), ("reflectance", C.c_float),
                ("A", C.c_float), ("B", C.c_float), ("C", C.c_float)]


class rr_bvh_options(C.Structure):
    _fields_ = [("max_leaf_size", C.c_uint32), ("sah_bins", C.c_uint32),
                ("n_threads", C.c_uint32), ("split_pct", C.c_uint32), ("width", C.c_uint32),
                ("merge_leaves", C.c_uint32), ("builder", C.c_uint32), ("collapse", C.c_uint32),
                ("spatial_pct", C.c_int32)]


class rr_bvh_info(C.Structure):
    _fields_ = [("n_tris", C.c_uint32), ("n_hittable", C.c_uint32), ("n_nodes", C.c_uint32),
                ("n_leaves", C.c_uint32), ("max_depth", C.c_uint32), ("max_stack", C.c_uint32),
                ("device_bytes", C.c_uint64), ("sah_cost", C.c_double), ("build_ms", C.c_double)]


class rr_scan_stats(C.Structure):
    _fields_ = [("segments", C.c_uint64), ("rays_per_depth", C.c_uint64 * RR_MAX_BOUNCES),
                ("overflow", C.c_uint32), ("air_rays", C.c_uint32)]


class rr_profile(C.Structure):
    _fields_ = [("trace_launches", C.c_uint64), ("trace_ms", C.c_double),
                ("trace_level_ms", C.c_double * RR_MAX_BOUNCES), ("shade_ms", C.c_double),
                ("raygen_ms", C.c_double), ("node_visits", C.c_uint64),
                ("tri_tests", C.c_uint64), ("rays", C.c_uint64), ("hits", C.c_uint64),
                ("wave_iters", C.c_uint64 * RR_MAX_BOUNCES),
                ("active_lanes", C.c_uint64 * RR_MAX_BOUNCES),
                ("tail_wave_iters", C.c_uint64 * RR_MAX_BOUNCES),
                ("tail_active_lanes", C.c_uint64 * RR_MAX_BOUNCES),
                ("max_ray_iters", C.c_uint64 * RR_MAX_BOUNCES), ("shadow_ms", C.c_double)]


RR_PROFILE_TIME, RR_PROFILE_COUNT, RR_PROFILE_TRACE_TIME = 1, 2, 4


class rr_tuning(C.Structure):
    _fields_ = [("refill_lanes", C.c_uint32), ("trace_waves_per_cu", C.c_uint32),
                ("pool_rays", C.c_uint32), ("batch_budget_mb", C.c_uint32),
                ("tri_batch", C.c_uint32), ("fused", C.c_uint32), ("shade_batch", C.c_uint32),
                ("tail_help", C.c_uint32)]


class rr_server_options(C.Structure):
    _fields_ = [("n_slots", C.c_uint32), ("max_batch_scans", C.c_uint32),
                ("memory_budget", C.c_uint64), ("reserved", C.c_uint32 * 4)]


class rr_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("rejected", C.c_uint64),
                ("batches", C.c_uint64), ("segments", C.c_uint64),
                ("latency_p50_ms", C.c_double), ("latency_p99_ms", C.c_double),
                ("latency_mean_ms", C.c_double), ("latency_max_ms", C.c_double),
                ("wall_s", C.c_double), ("scans_per_s", C.c_double), ("mseg_per_s", C.c_double)]


class rr_scan_desc(C.Structure):
    _fields_ = [("pose", rr_pose), ("params", rr_sensor_params), ("image_dev", C.c_void_p),
                ("primary_mask_dev", C.c_void_p)]


class rr_post_params(C.Structure):
    _fields_ = [("blur_sigma_bins", C.c_float), ("uniform_amp", C.c_float), ("perlin_amp", C.c_float),
                ("perlin_cell_az", C.c_float), ("perlin_cell_bins", C.c_float), ("db_floor", C.c_float),
                ("max_value", C.c_uint32), ("reserved0", C.c_uint32), ("seed", C.c_uint64),
                ("scan_id", C.c_uint32), ("reserved1", C.c_uint32)]


EXPORTS = (
    "rr_status_str", "rr_create", "rr_destroy", "rr_last_error", "rr_scene_upload",
    "rr_bvh_build", "rr_bvh_get_info", "rr_bvh_selfcheck", "rr_scene_release",
    "rr_workspace_query", "rr_radar_scan", "rr_radar_scan_ws", "rr_radar_scan_records",
    "rr_radar_scan_batch", "rr_batch_workspace_query", "rr_profile_enable", "rr_profile_read",
    "rr_set_tuning", "rr_get_tuning", "rr_server_create", "rr_server_submit", "rr_server_wait",
    "rr_server_poll", "rr_server_get_stats", "rr_server_reset_stats", "rr_server_destroy",
    "rr_autotune", "rr_graph_create", "rr_graph_launch", "rr_graph_destroy", "rr_measure_gather",
    "rr_postprocess", "rr_radar_scan_post", "rr_bvh_refit", "rr_radar_scan_noalloc", "rr_scratch_bytes",
    "rr_autotune_batch",
)

_lib = None


def load_library():
    """Load libradarays_hip.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    # Load PyTorch first: the library's libamdhip64 dependency then resolves
    # (by soname) to the HIP runtime torch has already loaded, so the two
    # share one runtime.  Loaded the other way round, torch later finds no
    # device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2310_03505_amd.build` (there is no fallback)")
    lib = C.CDLL(LIB_PATH)
    P, vp = C.POINTER, C.c_void_p
    st = C.c_int32
    sig = {
        "rr_status_str": (C.c_char_p, [st]),
        "rr_create": (st, [C.c_int, P(vp)]),
        "rr_destroy": (st, [vp]),
        "rr_last_error": (C.c_char_p, [vp]),
        "rr_scene_upload": (st, [vp, P(C.c_float), C.c_uint32, P(C.c_uint32), C.c_uint32,
                                 P(C.c_uint16), P(vp)]),
        "rr_bvh_build": (st, [vp, vp, P(rr_bvh_options)]),
        "rr_bvh_get_info": (st, [vp, P(rr_bvh_info)]),
        "rr_bvh_selfcheck": (st, [vp, C.c_uint32, C.c_uint64, P(C.c_uint64)]),
        "rr_scene_release": (st, [vp, vp]),
        "rr_workspace_query": (st, [P(rr_sensor_params), P(C.c_size_t)]),
        "rr_radar_scan": (st, [vp, vp, P(rr_pose), P(rr_sensor_params), P(rr_material), C.c_uint32,
                               vp, P(rr_scan_stats), vp]),
        "rr_radar_scan_ws": (st, [vp, vp, P(rr_pose), P(rr_sensor_params), P(rr_material),
                                  C.c_uint32, vp, vp, C.c_size_t, P(rr_scan_stats), vp]),
        "rr_radar_scan_noalloc": (st, [vp, vp, P(rr_pose), P(rr_sensor_params), P(rr_material),
                                       C.c_uint32, vp, P(rr_scan_stats), vp]),
        "rr_scratch_bytes": (st, [P(C.c_size_t)]),
        "rr_radar_scan_records": (st, [vp, vp, P(rr_pose), P(rr_sensor_params), P(rr_material),
                                       C.c_uint32, vp, vp, vp, vp, P(rr_scan_stats), vp]),
        "rr_radar_scan_batch": (st, [vp, vp, P(rr_scan_desc), C.c_uint32, P(rr_material),
                                     C.c_uint32, P(rr_scan_stats), vp]),
        "rr_batch_workspace_query": (st, [P(rr_scan_desc), C.c_uint32, P(C.c_size_t)]),
        "rr_profile_enable": (st, [vp, C.c_uint32]),
        "rr_profile_read": (st, [vp, P(rr_profile)]),
        "rr_set_tuning": (st, [vp, P(rr_tuning)]),
        "rr_get_tuning": (st, [vp, P(rr_tuning)]),
        "rr_server_create": (st, [vp, vp, P(rr_material), C.c_uint32, P(rr_server_options), P(vp)]),
        "rr_server_submit": (st, [vp, P(rr_pose), P(rr_sensor_params), vp, P(C.c_uint64)]),
        "rr_server_wait": (st, [vp, C.c_uint64, P(C.c_double)]),
        "rr_server_poll": (st, [vp, C.c_uint64, P(C.c_int), P(C.c_double)]),
        "rr_server_get_stats": (st, [vp, P(rr_server_stats)]),
        "rr_server_reset_stats": (st, [vp]),
        "rr_server_destroy": (st, [vp]),
        "rr_autotune": (st, [vp, vp, P(rr_pose), P(rr_sensor_params), P(rr_material), C.c_uint32,
                             vp, C.c_uint32, P(rr_tuning), P(C.c_double), vp]),
        "rr_autotune_batch": (st, [vp, vp, P(rr_scan_desc), C.c_uint32, P(rr_material), C.c_uint32,
                                   C.c_uint32, P(rr_tuning), P(C.c_double), vp]),
        "rr_graph_create": (st, [vp, vp, P(rr_scan_desc), C.c_uint32, P(rr_material), C.c_uint32,
                                 P(vp)]),
        "rr_graph_launch": (st, [vp, P(rr_scan_desc), vp]),
        "rr_graph_destroy": (st, [vp]),
        "rr_measure_gather": (st, [vp, C.c_uint64, C.c_uint32, P(C.c_double)]),
        "rr_bvh_refit": (st, [vp, vp, vp, C.c_uint32, vp]),
        "rr_postprocess": (st, [vp, vp, C.c_uint32, C.c_uint32, C.c_uint32, P(rr_post_params), vp, vp, vp]),
        "rr_radar_scan_post": (st, [vp, vp, P(rr_pose), P(rr_sensor_params), P(rr_material), C.c_uint32,
                                    P(rr_post_params), vp, vp, vp, P(rr_scan_stats), vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(status: int, ctx=None):
    if status != RR_OK:
        lib = load_library()
        msg = lib.rr_last_error(ctx).decode(errors="replace")
        raise RadarError(status, msg or lib.rr_status_str(status).decode())


# ------------------------------------------------------------------ marshalling
def make_pose(pose: dict) -> rr_pose:
    return rr_pose((C.c_float * 3)(*pose["position"]), (C.c_float * 4)(*pose["quat_wxyz"]))


def make_params(p: dict) -> rr_sensor_params:
    return rr_sensor_params(p["n_azimuth"], p["rays_per_beam"], p["max_bounces"], p["n_bins"],
                            p["bin_size_m"], p["beam_width_rad"], p["beam_prob"],
                            p["energy_cutoff"], p["seed"], p["scan_id"], p["flags"],
                            p.get("beam_stretch_az", 0.0), p.get("beam_stretch_inc", 0.0))


def make_materials(mats):
    arr = (rr_material * max(1, len(mats)))()
    for i, m in enumerate(mats):
        arr[i] = rr_material(m["kind"], m["n"], m["reflectance"], m["A"], m["B"], m["C"])
    return arr


def _stream_handle(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ the C ABI, by name
def rr_create(device: int = 0):
    lib = load_library()
    h = C.c_void_p()
    _check(lib.rr_create(device, C.byref(h)))
    return h


def rr_destroy(ctx):
    _check(load_library().rr_destroy(ctx))


def rr_scene_upload(ctx, vertices, indices, tri_material):
    import numpy as np
    lib = load_library()
    V = np.ascontiguousarray(vertices, dtype=np.float32)
    F = np.ascontiguousarray(indices, dtype=np.uint32)
    M = np.ascontiguousarray(tri_material, dtype=np.uint16)
    h = C.c_void_p()
    _check(lib.rr_scene_upload(ctx, V.ctypes.data_as(C.POINTER(C.c_float)), V.shape[0],
                               F.ctypes.data_as(C.POINTER(C.c_uint32)), F.shape[0],
                               M.ctypes.data_as(C.POINTER(C.c_uint16)), C.byref(h)), ctx)
    return h


def rr_bvh_build(ctx, scene, max_leaf_size: int = 0, sah_bins: int = 0, n_threads: int = 0,
                 split_pct: int = 0, width: int = 0, merge_leaves: int = 0, builder: int = 0,
                 collapse: int = 0, spatial_pct: int = 0):
    """builder 0: binned SAH on the host; 1: linear BVH on the GPU.
    collapse (host builder, four-wide): 0 default (cost-optimal), 1 greedy,
    2 cost-optimal.  spatial_pct (host builder): spatial-split budget in
    percent of the triangles, 0 default (10), -1 none."""
    opt = rr_bvh_options(max_leaf_size, sah_bins, n_threads, split_pct, width, merge_leaves, builder,
                         collapse, spatial_pct)
    _check(load_library().rr_bvh_build(ctx, scene, C.byref(opt)), ctx)


def rr_bvh_refit(ctx, scene, vertices, stream=None):
    """New vertex positions (a float32 CUDA tensor [nv, 3]) for a scene with
    a four-wide BVH (either builder); the tree is refitted on the GPU,
    stream-ordered."""
    import torch
    if vertices.dtype != torch.float32 or not vertices.is_contiguous() or vertices.dim() != 2:
        raise ValueError("vertices must be a contiguous float32 tensor [nv, 3]")
    _check(load_library().rr_bvh_refit(ctx, scene, _ptr(vertices), vertices.shape[0], _stream_handle(stream)), ctx)


def rr_bvh_get_info(scene) -> dict:
    info = rr_bvh_info()
    _check(load_library().rr_bvh_get_info(scene, C.byref(info)))
    return {k: getattr(info, k) for k, _ in rr_bvh_info._fields_ if k != "reserved"}


def rr_bvh_selfcheck(scene, n_rays: int = 10000, seed: int = 1) -> int:
    out = C.c_uint64()
    _check(load_library().rr_bvh_selfcheck(scene, n_rays, seed, C.byref(out)))
    return int(out.value)


def rr_scene_release(ctx, scene):
    _check(load_library().rr_scene_release(ctx, scene), ctx)


def rr_workspace_query(params: dict) -> int:
    out = C.c_size_t()
    prm = make_params(params)
    _check(load_library().rr_workspace_query(C.byref(prm), C.byref(out)))
    return int(out.value)


def _stats_dict(st: rr_scan_stats) -> dict:
    return dict(segments=int(st.segments), rays_per_depth=[int(x) for x in st.rays_per_depth],
                overflow=int(st.overflow), air_rays=int(st.air_rays))


def rr_radar_scan(ctx, scene, pose: dict, params: dict, materials, image=None, stats=False,
                  stream=None):
    """One polar image into ``image`` (a float32 CUDA tensor [n_az, n_bins],
    allocated if None).  Returns (image, stats-or-None)."""
    import torch
    if image is None:
        image = torch.empty((params["n_azimuth"], params["n_bins"]), dtype=torch.float32,
                            device="cuda")
    st = rr_scan_stats() if stats else None
    mats = make_materials(materials)
    pr, ps = make_pose(pose), make_params(params)
    _check(load_library().rr_radar_scan(ctx, scene, C.byref(pr), C.byref(ps), mats, len(materials),
                                        _ptr(image), C.byref(st) if st is not None else None,
                                        _stream_handle(stream)), ctx)
    return image, (_stats_dict(st) if st is not None else None)


def rr_radar_scan_ws(ctx, scene, pose: dict, params: dict, materials, image, workspace,
                     stats=False, stream=None):
    st = rr_scan_stats() if stats else None
    mats = make_materials(materials)
    pr, ps = make_pose(pose), make_params(params)
    _check(load_library().rr_radar_scan_ws(ctx, scene, C.byref(pr), C.byref(ps), mats,
                                           len(materials), _ptr(image), _ptr(workspace),
                                           workspace.numel() * workspace.element_size(),
                                           C.byref(st) if st is not None else None,
                                           _stream_handle(stream)), ctx)
    return image, (_stats_dict(st) if st is not None else None)


def rr_radar_scan_noalloc(ctx, scene, pose: dict, params: dict, materials, image, stats=False, stream=None):
    """rr_radar_scan on the library's fixed scratch array: no device allocation
    (the caller passes the output image)."""
    st = rr_scan_stats() if stats else None
    mats = make_materials(materials)
    pr, ps = make_pose(pose), make_params(params)
    _check(load_library().rr_radar_scan_noalloc(ctx, scene, C.byref(pr), C.byref(ps), mats,
                                                len(materials), _ptr(image),
                                                C.byref(st) if st is not None else None,
                                                _stream_handle(stream)), ctx)
    return image, (_stats_dict(st) if st is not None else None)


def rr_scratch_bytes() -> int:
    out = C.c_size_t()
    _check(load_library().rr_scratch_bytes(C.byref(out)))
    return int(out.value)


def rr_radar_scan_records(ctx, scene, pose: dict, params: dict, materials, primary_mask=None,
                          records=True, accum=True, stats=True, stream=None):
    """Debug/parity scan.  Returns dict(image, records, accum, stats) with
    CUDA tensors (records int32 [N_p, 2^B-1], accum int64 view of the uint64
    fixed-point accumulator); with RR_AIR_PATH also air_records int32
    [N_p, 2^B-1], the air-path outcome of each hit (-2 none, 0 returned,
    1 blocked, 2 beyond the last bin)."""
    import torch
    n_az, n_s, nb, B = (params["n_azimuth"], params["rays_per_beam"], params["n_bins"],
                        params["max_bounces"])
    nheap = (1 << B) - 1
    air = bool(params.get("flags", 0) & RR_AIR_PATH)
    image = torch.empty((n_az, nb), dtype=torch.float32, device="cuda")
    rec = torch.empty((n_az * n_s, 2 * nheap if air else nheap), dtype=torch.int32,
                      device="cuda") if records else None
    acc = torch.empty((n_az, nb), dtype=torch.int64, device="cuda") if accum else None
    st = rr_scan_stats() if stats else None
    mats = make_materials(materials)
    pr, ps = make_pose(pose), make_params(params)
    _check(load_library().rr_radar_scan_records(
        ctx, scene, C.byref(pr), C.byref(ps), mats, len(materials), _ptr(primary_mask),
        _ptr(image), _ptr(rec), _ptr(acc), C.byref(st) if st is not None else None,
        _stream_handle(stream)), ctx)
    out = dict(image=image, records=rec, accum=acc, stats=_stats_dict(st) if st is not None else None)
    if rec is not None and air:
        out["records"], out["air_records"] = rec[:, :nheap], rec[:, nheap:]
    return out


def make_scan_descs(scans, images, masks=None):
    """masks: optional list of uint8 device tensors (or None) per scan."""
    arr = (rr_scan_desc * len(scans))()
    for i, ((pose, params), img) in enumerate(zip(scans, images)):
        m = masks[i] if masks is not None else None
        arr[i] = rr_scan_desc(make_pose(pose), make_params(params), C.c_void_p(img.data_ptr()),
                              C.c_void_p(m.data_ptr()) if m is not None else None)
    return arr


def rr_batch_workspace_query(scans) -> int:
    arr = (rr_scan_desc * len(scans))()
    for i, (pose, params) in enumerate(scans):
        arr[i] = rr_scan_desc(make_pose(pose), make_params(params), None, None)
    out = C.c_size_t()
    _check(load_library().rr_batch_workspace_query(arr, len(scans), C.byref(out)))
    return int(out.value)


def rr_radar_scan_batch(ctx, scene, scans, materials, images=None, stats=False, stream=None,
                        masks=None):
    """Many (pose, params) scans in one pass.  Returns (images, stats).
    masks: optional per-scan uint8 device tensors of n_azimuth * rays_per_beam
    (None entries trace every primary)."""
    import torch
    if images is None:
        images = [torch.empty((p["n_azimuth"], p["n_bins"]), dtype=torch.float32, device="cuda")
                  for _, p in scans]
    descs = make_scan_descs(scans, images, masks)
    st = rr_scan_stats() if stats else None
    mats = make_materials(materials)
    _check(load_library().rr_radar_scan_batch(ctx, scene, descs, len(scans), mats, len(materials),
                                              C.byref(st) if st is not None else None,
                                              _stream_handle(stream)), ctx)
    return images, (_stats_dict(st) if st is not None else None)


TUNING_KEYS = ("refill_lanes", "trace_waves_per_cu", "pool_rays", "batch_budget_mb", "tri_batch",
               "fused", "shade_batch", "tail_help")
RR_TAIL_HELP_OFF = 0xFFFFFFFF


def _tuning_dict(t) -> dict:
    return {k: int(getattr(t, k)) for k in TUNING_KEYS}


def rr_set_tuning(ctx, refill_lanes: int = 0, trace_waves_per_cu: int = 0, pool_rays: int = 0,
                  batch_budget_mb: int = 0, tri_batch: int = 0, fused: int = 0,
                  shade_batch: int = 0, tail_help: int = 0):
    t = rr_tuning(refill_lanes, trace_waves_per_cu, pool_rays, batch_budget_mb, tri_batch, fused,
                  shade_batch, tail_help)
    _check(load_library().rr_set_tuning(ctx, C.byref(t)), ctx)


def rr_get_tuning(ctx) -> dict:
    t = rr_tuning()
    _check(load_library().rr_get_tuning(ctx, C.byref(t)), ctx)
    return _tuning_dict(t)


def rr_autotune(ctx, scene, pose: dict, params: dict, materials, image=None, reps: int = 5,
                stream=None):
    """Times candidate launch parameters on this scan and keeps the fastest.
    Returns (tuning dict, ms per scan)."""
    import torch
    if image is None:
        image = torch.empty((params["n_azimuth"], params["n_bins"]), dtype=torch.float32,
                            device="cuda")
    t = rr_tuning()
    ms = C.c_double()
    mats = make_materials(materials)
    _check(load_library().rr_autotune(ctx, scene, C.byref(make_pose(pose)),
                                      C.byref(make_params(params)), mats, len(materials),
                                      _ptr(image), reps, C.byref(t), C.byref(ms),
                                      _stream_handle(stream)), ctx)
    return _tuning_dict(t), float(ms.value)


def rr_autotune_batch(ctx, scene, scans, materials, images=None, reps: int = 2, stream=None):
    """Times candidate launch parameters on rr_radar_scan_batch over these
    (pose, params) scans and keeps the fastest.  Returns (tuning dict, ms per
    batch)."""
    import torch
    if images is None:
        images = [torch.empty((p["n_azimuth"], p["n_bins"]), dtype=torch.float32, device="cuda")
                  for _, p in scans]
    descs = make_scan_descs(scans, images)
    t = rr_tuning()
    ms = C.c_double()
    mats = make_materials(materials)
    _check(load_library().rr_autotune_batch(ctx, scene, descs, len(scans), mats, len(materials), reps,
                                            C.byref(t), C.byref(ms), _stream_handle(stream)), ctx)
    return _tuning_dict(t), float(ms.value)


def rr_graph_create(ctx, scene, scans, materials, images=None, masks=None):
    """Captures the launch sequence of these (pose, params) scans.  Returns
    (graph handle, images); the images stay the graph's outputs until a
    launch passes others."""
    import torch
    if images is None:
        images = [torch.empty((p["n_azimuth"], p["n_bins"]), dtype=torch.float32, device="cuda")
                  for _, p in scans]
    descs = make_scan_descs(scans, images, masks)
    mats = make_materials(materials)
    h = C.c_void_p()
    _check(load_library().rr_graph_create(ctx, scene, descs, len(scans), mats, len(materials),
                                          C.byref(h)), ctx)
    return h, images


def rr_graph_launch(graph, scans=None, images=None, stream=None, masks=None):
    """Replays the graph; with scans (and their images) the per-scan tables are
    replaced first."""
    if scans is not None and images is None:
        raise ValueError("new scans need their output images")
    descs = make_scan_descs(scans, images, masks) if scans is not None else None
    _check(load_library().rr_graph_launch(graph, descs, _stream_handle(stream)))


def rr_graph_destroy(graph):
    _check(load_library().rr_graph_destroy(graph))


def rr_measure_gather(ctx, working_set_bytes: int, reads_mb: int = 4096) -> float:
    """Random 64-byte gather rate (GB/s) over a device working set."""
    out = C.c_double()
    _check(load_library().rr_measure_gather(ctx, working_set_bytes, reads_mb, C.byref(out)), ctx)
    return float(out.value)


def rr_profile_enable(ctx, flags: int):
    _check(load_library().rr_profile_enable(ctx, flags), ctx)


def rr_profile_read(ctx) -> dict:
    p = rr_profile()
    _check(load_library().rr_profile_read(ctx, C.byref(p)), ctx)
    return dict(trace_launches=int(p.trace_launches), trace_ms=float(p.trace_ms),
                trace_level_ms=[float(x) for x in p.trace_level_ms], shade_ms=float(p.shade_ms),
                raygen_ms=float(p.raygen_ms), node_visits=int(p.node_visits),
                tri_tests=int(p.tri_tests), rays=int(p.rays), hits=int(p.hits),
                wave_iters=list(p.wave_iters), active_lanes=list(p.active_lanes),
                tail_wave_iters=list(p.tail_wave_iters),
                tail_active_lanes=list(p.tail_active_lanes),
                max_ray_iters=list(p.max_ray_iters), shadow_ms=float(p.shadow_ms))


def rr_server_create(ctx, scene, materials, n_slots: int = 0, max_batch_scans: int = 0,
                     memory_budget: int = 0):
    opt = rr_server_options(n_slots, max_batch_scans, memory_budget)
    mats = make_materials(materials)
    h = C.c_void_p()
    _check(load_library().rr_server_create(ctx, scene, mats, len(materials), C.byref(opt),
                                           C.byref(h)), ctx)
    return h


def rr_server_submit(srv, pose: dict, params: dict, image) -> int:
    t = C.c_uint64()
    pr, ps = make_pose(pose), make_params(params)
    _check(load_library().rr_server_submit(srv, C.byref(pr), C.byref(ps), _ptr(image), C.byref(t)))
    return int(t.value)


def rr_server_wait(srv, ticket: int) -> float:
    lat = C.c_double()
    _check(load_library().rr_server_wait(srv, ticket, C.byref(lat)))
    return float(lat.value)


def rr_server_poll(srv, ticket: int):
    done, lat = C.c_int(), C.c_double()
    _check(load_library().rr_server_poll(srv, ticket, C.byref(done), C.byref(lat)))
    return bool(done.value), float(lat.value)


def rr_server_get_stats(srv) -> dict:
    st = rr_server_stats()
    _check(load_library().rr_server_get_stats(srv, C.byref(st)))
    return {k: getattr(st, k) for k, _ in rr_server_stats._fields_}


def rr_server_reset_stats(srv):
    _check(load_library().rr_server_reset_stats(srv))


def rr_server_destroy(srv):
    _check(load_library().rr_server_destroy(srv))


# ------------------------------------------------------------------ epilogue
POST_DEFAULTS = dict(blur_sigma_bins=0.0, uniform_amp=0.0, perlin_amp=0.0, perlin_cell_az=16.0,
                     perlin_cell_bins=64.0, db_floor=-100.0, max_value=255, seed=0x5EED, scan_id=0)


def make_post(post: dict) -> rr_post_params:
    unknown = set(post) - set(POST_DEFAULTS)
    if unknown:
        raise ValueError(f"unknown epilogue parameters: {sorted(unknown)}")
    q = dict(POST_DEFAULTS, **post)
    return rr_post_params(q["blur_sigma_bins"], q["uniform_amp"], q["perlin_amp"], q["perlin_cell_az"],
                          q["perlin_cell_bins"], q["db_floor"], q["max_value"], 0, q["seed"], q["scan_id"], 0)


def rr_postprocess(ctx, images, post: dict, db=None, u8=None, want_db=True, want_u8=True, stream=None):
    """Epilogue of float32 CUDA images [n_az, n_bins] or [n_images, n_az,
    n_bins] (contiguous).  Returns (db, u8); outputs are allocated when None
    and wanted."""
    import torch
    if images.dtype != torch.float32 or not images.is_contiguous() or images.dim() not in (2, 3):
        raise ValueError("images must be a contiguous float32 tensor of 2 or 3 dimensions")
    shape = images.shape
    n_img, n_az, n_bins = (1, *shape) if images.dim() == 2 else shape
    if db is None and want_db:
        db = torch.empty(shape, dtype=torch.float32, device=images.device)
    if u8 is None and want_u8:
        u8 = torch.empty(shape, dtype=torch.uint8, device=images.device)
    for t, dt in ((db, torch.float32), (u8, torch.uint8)):
        if t is not None and (t.dtype != dt or t.shape != shape or not t.is_contiguous()):
            raise ValueError("outputs must be contiguous, of the images' shape, float32 (dB) and uint8")
    pp = make_post(post)
    _check(load_library().rr_postprocess(ctx, _ptr(images), n_img, n_az, n_bins, C.byref(pp), _ptr(db),
                                         _ptr(u8), _stream_handle(stream)), ctx)
    return db, u8


def rr_radar_scan_post(ctx, scene, pose: dict, params: dict, materials, post: dict, image=None, db=None,
                       u8=None, want_image=True, want_db=True, want_u8=True, stats=False, stream=None):
    """rr_radar_scan with the epilogue fused into its last launch.  Returns
    (image, db, u8, stats-or-None)."""
    import torch
    shape = (params["n_azimuth"], params["n_bins"])
    if image is None and want_image:
        image = torch.empty(shape, dtype=torch.float32, device="cuda")
    if db is None and want_db:
        db = torch.empty(shape, dtype=torch.float32, device="cuda")
    if u8 is None and want_u8:
        u8 = torch.empty(shape, dtype=torch.uint8, device="cuda")
    st = rr_scan_stats() if stats else None
    mats = make_materials(materials)
    pr, ps, pp = make_pose(pose), make_params(params), make_post(post)
    _check(load_library().rr_radar_scan_post(ctx, scene, C.byref(pr), C.byref(ps), mats, len(materials),
                                             C.byref(pp), _ptr(image), _ptr(db), _ptr(u8),
                                             C.byref(st) if st is not None else None,
                                             _stream_handle(stream)), ctx)
    return image, db, u8, (_stats_dict(st) if st is not None else None)


# ------------------------------------------------------------------ convenience
class Context:
    def __init__(self, device: int = 0):
        self.handle = rr_create(device)

    def close(self):
        if self.handle:
            rr_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Scene:
    """A mesh resident on the GPU with its BVH built."""

    def __init__(self, ctx: Context | None, vertices, indices, tri_material, build=True, **bvh_opts):
        self.ctx = ctx
        self._c = ctx.handle if ctx is not None else None
        self.handle = rr_scene_upload(self._c, vertices, indices, tri_material)
        if build:
            rr_bvh_build(self._c, self.handle, **bvh_opts)

    def info(self) -> dict:
        return rr_bvh_get_info(self.handle)

    def refit(self, vertices, stream=None):
        rr_bvh_refit(self._c, self.handle, vertices, stream)

    def selfcheck(self, n_rays=10000, seed=1) -> int:
        return rr_bvh_selfcheck(self.handle, n_rays, seed)

    def release(self):
        if self.handle:
            rr_scene_release(self._c, self.handle)
            self.handle = None


def scan(scene: Scene, pose: dict, params: dict, materials, image=None, stream=None):
    """One polar image of a resident scene (a Scene built with a context) on
    the current stream, or `stream`: the float32 [n_azimuth, n_bins] CUDA
    tensor (rr_radar_scan through the scene's context)."""
    if scene.ctx is None or not scene.handle:
        raise ValueError("the scene has no device copy (built without a context, or released)")
    img, _ = rr_radar_scan(scene._c, scene.handle, pose, params, materials, image=image, stream=stream)
    return img
