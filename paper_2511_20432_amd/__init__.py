"""MI355X (gfx950) implementation of the semi-analytical isogeometric thermal
model for laser powder bed fusion.

  workloads  seeded input generators (patches, materials, scan paths)
  sa_iga     ctypes binding of the HIP library libsa_iga.so (include/sa_iga.h)
  build      in-tree hipcc build of the library
"""
from . import workloads  # noqa: F401

__all__ = ["workloads"]
