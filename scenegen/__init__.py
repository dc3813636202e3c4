"""Seeded synthetic scenes for shortest-path-map builds.

This package only *constructs* inputs: polygonal obstacles, point sources and
segment sources on an integer domain.  It holds none of the shortest-path-map
arithmetic (no visibility, no distances, no propagation); both the CPU oracle
and the GPU library consume its output.
"""
from .scenes import (  # noqa: F401
    Scene,
    config1,
    config2,
    config3,
    config4_list,
    config5_agents,
    random_small,
    profiling_grid,
    scene_from_arrays,
    load_scene,
    save_scene,
)
