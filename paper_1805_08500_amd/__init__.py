"""MI355X-native shortest path maps (Farias & Kallmann, "Improved Shortest
Path Maps with GPU Shaders"): a HIP library behind a C ABI (include/spm.h)
and a thin PyTorch-facing binding."""
from . import _lib  # noqa: F401
from .spm import (  # noqa: F401
    BatchBuilder,
    Builder,
    Graph,
    SPMDistance,
    DeviceScene,
    Map,
    Timer,
    agent_distance,
    build,
    query_path,
    query_points,
    query_sizes,
    source_gradients,
    validate,
)
