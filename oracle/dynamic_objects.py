"""Oracle of the N_D feature of the state vector (test infrastructure only).

What is computed (paper §III-D, State Representation; Table IV; the
environment vector E_t of §IV-C, Eq. 1): N_D, the number of dynamic objects
in the frame. The renderer's custom stencil buffer marks the pixels of
dynamic objects, and the paper finds the objects by clustering that buffer;
it names no clustering method.

Readings taken here:

* A pixel belongs to a dynamic object iff its stencil value is non-zero.
* An object is a connected component of such pixels: two marked pixels are
  in one object iff a chain of marked pixels joins them, each adjacent to
  the next. Adjacency is 8-connectivity by default (pixels sharing an edge
  or a corner: a diagonal touch joins two rasterised objects), or
  4-connectivity (an edge) on request.
* N_D of a frame is the number of its components. Objects that touch or
  overlap in the frame count once, as one cluster.

The library step is scipy.ndimage.label with the 3 x 3 structuring element
of the chosen connectivity; the pins check it against a flood fill written
out in the tests, closed forms and planted mistakes. Nothing here is shared
with, or imported by, the HIP path.
"""

from __future__ import annotations

import numpy as np
from scipy import ndimage

CONNECTIVITY = (4, 8)


def structure(connectivity: int) -> np.ndarray:
    """The 3 x 3 neighbourhood of a pixel under the given connectivity."""
    if connectivity == 4:
        return np.array([[0, 1, 0], [1, 1, 1], [0, 1, 0]], dtype=bool)
    if connectivity == 8:
        return np.ones((3, 3), dtype=bool)
    raise ValueError("connectivity is 4 or 8")


def frame_objects(stencil: np.ndarray, connectivity: int = 8) -> int:
    """N_D of one frame: stencil [H, W] (any integer or bool dtype)."""
    mask = np.asarray(stencil) != 0
    if mask.ndim != 2:
        raise ValueError("a frame's stencil is [H, W]")
    _, count = ndimage.label(mask, structure=structure(connectivity))
    return int(count)


def dynamic_objects(stencil: np.ndarray, connectivity: int = 8) -> np.ndarray:
    """N_D of every frame of stencil [N, H, W]: int64 [N]."""
    stencil = np.asarray(stencil)
    if stencil.ndim != 3:
        raise ValueError("dynamic_objects takes a [N, H, W] stencil")
    return np.array([frame_objects(f, connectivity) for f in stencil], dtype=np.int64)
