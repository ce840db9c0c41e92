"""MI355X (gfx950) rendering hot path of SuperCaustics (arXiv 2107.11008).

The HIP library ``libsc.so`` (C ABI in ``include/sc.h``) renders the
paper's outputs for scenes with transparent objects: the spectral image with
refraction, dispersion and caustics, depth, normals and the object mask,
plus the photon caustic map.  ``Context`` / ``Bvh`` in ``_sc`` are the thin
Python binding (argument marshalling only).
"""
from ._sc import Batch, Bvh, Context, PhotonMap, ScError, UNet, autotune_batch, load  # noqa: F401

__all__ = ["Context", "Bvh", "Batch", "PhotonMap", "UNet", "ScError", "autotune_batch", "load"]
