"""MI355X-native preconditioned MINRES for symmetrised BLTT all-at-once systems.

Modules:
  bltt       ctypes binding of libbltt.so (the HIP solver)
  workloads  seeded synthetic problem descriptions
  build_lib  in-tree build of libbltt.so for gfx950
"""
