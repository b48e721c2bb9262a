"""MI355X (gfx950) implementation of the soft/affine incremental-potential-contact
Newton step (HIP kernels behind the C interface of include/zema.h)."""
from .zema import Scene, ZemaError, lib, scene_create  # noqa: F401
