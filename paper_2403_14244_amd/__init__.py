"""MI355X (gfx950) rasterizer for isotropic Gaussian splatting (arXiv 2403.14244).

The hot path (projection, tile binning, radix sort, compositing and its backward) runs
in hand-written HIP kernels behind the C ABI of include/isogs.h; this package is the
thin binding. Importing it loads the in-tree library and fails if it is not built.
"""
from ._abi import lib as _lib, IsoGSError  # noqa: F401

_lib()

from .rasterizer import (GaussianScene, Footprints, TileBins, Rasterizer, IsoGSRender,  # noqa: E402,F401
                         split_images, tiles_of)
from .field2d import (Field2DRenderer, Field2DRender, Field2DAnisoRenderer, Field2DAnisoRender,  # noqa: E402,F401
                      tree_init, prune, split, merge, octree_init)
from .loss import SSIM, L1, ssim, l1_loss, l1_ssim_loss  # noqa: E402,F401
from .aniso import AnisoGaussianScene, AnisoFootprints, AnisoRasterizer, AnisoGSRender  # noqa: E402,F401

__all__ = ["GaussianScene", "Footprints", "TileBins", "Rasterizer", "IsoGSRender", "IsoGSError",
           "split_images", "tiles_of", "Field2DRenderer", "Field2DRender", "SSIM", "L1", "ssim", "l1_loss", "l1_ssim_loss",
           "tree_init", "prune", "split", "merge", "octree_init", "Field2DAnisoRenderer", "Field2DAnisoRender", "AnisoGaussianScene", "AnisoFootprints", "AnisoRasterizer", "AnisoGSRender"]
