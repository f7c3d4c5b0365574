"""MI355X (gfx950) D2Q9 stream-and-collide with the collision models of Coreixas et al. (2020).

Submodules are imported lazily so that ``paper_2002_05265_amd.inputs`` can be used without
loading the HIP library:
  binding  - ctypes marshalling of the C ABI (liblbm.so, include/lbm.h)
  sim      - torch-facing wrapper (device memory and streams from torch)
  inputs   - seeded synthetic workloads
  build    - hipcc build of liblbm.so
"""
