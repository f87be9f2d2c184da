"""FP64 CPU oracle for the isotropic Gaussian splatting rasterizer.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``, never by the GPU library or its Python binding.
"""
from .isogs64 import *  # noqa: F401,F403
from .isogs64 import (ALPHA_MIN, ALPHA_MAX, T_MIN, TILE, RADIUS_GROW, RADIUS_PAD,  # noqa: F401
                      ALPHA_FLAG_REL, TERM_FLAG_REL)
from . import field2d64  # noqa: F401  (2D kernel-sum representation of Section 3)
from . import ssim64  # noqa: F401  (SSIM term of the loss)
from . import tree2d64  # noqa: F401  (quadtree initialisation, prune and split of 2D particles)
from . import aniso64  # noqa: F401  (anisotropic variant: eq. 5-7)
from . import octree64  # noqa: F401  (octree initialisation of 3D particles, merge of 2D particles)
from . import field2d_aniso64  # noqa: F401  (2D kernel sum with anisotropic kernels)
