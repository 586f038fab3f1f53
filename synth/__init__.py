"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks."""
from .scenes import (Workload, config1, config2, config3, config4_map, room_sequence, esdf_benchmark,
                     pinhole_dirs, lidar_dirs, make_pose, camera_rotation, multi_map_class,
                     MULTI_RES, MULTI_VOXEL, SEED_BASE, point_colors)
