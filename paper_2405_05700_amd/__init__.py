"""MI355X photon propagation through layered ice (the GPU stage of the
air-shower simulation chain of Meagher & van Santen).

* ``paper_2405_05700_amd.pp``: binding of the C-ABI library libpp.so
  (include/pp.h). Importing it raises if the library is not built.
* ``paper_2405_05700_amd.workloads``: seeded synthetic inputs.
* ``paper_2405_05700_amd.build``: builds libpp.so with hipcc for gfx950.
"""
__all__ = ["pp", "workloads", "build"]
