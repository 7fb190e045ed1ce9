"""MI355X-native block-adaptive ideal-MHD update (HIP kernels behind a C ABI, include/bmhd.h).

Modules:
  binding    ctypes binding of libbmhd.so (grid, set_state, fill_ghosts, reduce_dt, advance)
  workloads  seeded synthetic grids and initial states
  build      hipcc build of libbmhd.so for gfx950
"""
