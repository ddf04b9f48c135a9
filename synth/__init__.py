"""Seeded synthetic inputs shared by the product path and the oracle.

This package only draws random numbers and lays them out in the documented
input formats (primitive parameter arrays, camera descriptors, target images,
synthetic screen-space splat records).  It holds none of the rendering
method's arithmetic: no conditioning, projection, binning or compositing.
"""
from .scenes import (  # noqa: F401
    SceneSpec, ViewSpec, param_count, make_scene, make_view, look_at_view,
    make_target, make_config, CONFIG_NAMES, make_splat_records, make_elongated_records,
)
