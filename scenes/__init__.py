"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module only *generates inputs*: analytic scenes made of axis-aligned
boxes, ray-cast in float64 into pinhole depth maps with Gaussian noise added
in the disparity domain or into the returns of a spinning range scanner,
plus the sensor poses.  It contains none of the
fusion or regularisation arithmetic.  Both the FP64 oracle and the GPU
library consume exactly the arrays produced here.
"""
from .synth import (Camera, Frames, render_depth, scene_c1, scene_street,
                    frames_c1, frames_c2, frames_street, pose_translation,
                    pose_yaw, random_block_field, c4_block_counts, distance_to_scene,
                    inside_scene, scene_street, laser_scan)

__all__ = ["Camera", "Frames", "render_depth", "scene_c1", "scene_street",
           "frames_c1", "frames_c2", "frames_street", "pose_translation",
           "pose_yaw", "random_block_field", "c4_block_counts", "distance_to_scene", "inside_scene",
           "laser_scan"]
