"""Seeded synthetic inputs for the radar-scan path.

This package only builds inputs: triangle meshes, material tables, sensor
poses, sensor parameters, request streams and polar images for the
epilogue.  It holds none of the radar
method's arithmetic (no ray sampling, no intersection, no shading), so both
the CPU oracle and the HIP library can be fed from it without sharing any
code of the method.
"""
from .scenes import (  # noqa: F401
    FLAG_BEAM_GAIN, FLAG_FIXED_PATTERN, FLAG_MIRROR_PAIRS, FLAG_RETURN_ALL, FLAG_AIR_PATH,
    KIND_DIELECTRIC, KIND_METAL, KIND_LAMBERTIAN, KIND_COOK_TORRANCE,
    Scene, material_dielectric, material_metal, material_lambertian, material_cook_torrance,
    sensor_params, identity_pose, yaw_pose,
    tiny_room, urban_block, large_scene, empty_room, plane_scene, slab_scene,
    mirror_scene, single_triangle_scene, thin_pillars_scene,
    transform_scene,
)
from .poses import spline_poses, room_poses, request_stream, street_points  # noqa: F401
from .images import polar_images  # noqa: F401
