"""Seeded synthetic inputs for the motion-vector warp.

This package draws frames and motion-vector fields only. It contains none of
the warp's arithmetic, so both the CPU oracle and the HIP path can take their
inputs from it without sharing any part of the method.
"""

from .scenes import (  # noqa: F401
    CONFIGS,
    ConfigSpec,
    SinTexture,
    make_config,
    pan_rect_sequence,
    random_field_frames,
    quantize,
    upstream_gradient,
    world_position,
)
