"""Sub-element adaptive blended DG/FV scheme (arXiv:2011.03338) on MI355X.

* paper_2011_03338_amd.sedg      - ctypes binding of libsedg.so (HIP kernels, C ABI)
* paper_2011_03338_amd.workloads - seeded synthetic meshes and initial states
* paper_2011_03338_amd.build     - in-tree build of libsedg.so for gfx950
"""
