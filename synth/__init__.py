"""Seeded synthetic inputs shared by the renderer's tests, the benchmark and the oracle.

This package holds no step of the rendering method: it only draws voxel sets,
raw per-voxel parameters and sensor descriptions from seeded random number
generators.  Every function is deterministic given its seed.
"""
from .scenes import SceneData, config0_scene, config1_scene, config1_variant, single_voxel_scene, slab_scene, random_scene
from .sensors import (
    PINHOLE, FISHEYE_EQUIDISTANT, LIDAR_SPINNING,
    pinhole, fisheye_equidistant, lidar_spinning, look_at, yaw_pitch_camera, yaw_lidar,
    config0_camera, config1_camera, config2_lidar, random_rays,
)

__all__ = [
    "SceneData", "config0_scene", "config1_scene", "config1_variant", "single_voxel_scene", "slab_scene",
    "random_scene", "PINHOLE", "FISHEYE_EQUIDISTANT", "LIDAR_SPINNING", "pinhole", "fisheye_equidistant",
    "lidar_spinning", "look_at", "yaw_pitch_camera", "yaw_lidar", "config0_camera", "config1_camera",
    "config2_lidar", "random_rays",
]
