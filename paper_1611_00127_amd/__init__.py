"""MI355X (gfx950) solver library for the Newton Jacobian of fully implicit
two-phase porous-media flow, preconditioned by black-box AMG, CPR-AMG and
block factorisation (arXiv 1611.00127).

Modules:
  inputs  seeded synthetic workloads (no solver arithmetic)
  tpf     ctypes binding of the C ABI in include/tpf.h
  driver  torch-tensor plumbing around the binding (device buffers, streams)
  build   hipcc build of libtpf.so
"""
