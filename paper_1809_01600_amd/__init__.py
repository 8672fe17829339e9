"""MI355X-native LBM / Maxwell-Stefan solver (arXiv 1809.01600).

``paper_1809_01600_amd.lbm_ms``  - ctypes binding of liblbm_ms.so (the HIP library)
``paper_1809_01600_amd.inputs``  - seeded synthetic workloads
``paper_1809_01600_amd.build``   - hipcc build of the library
"""
