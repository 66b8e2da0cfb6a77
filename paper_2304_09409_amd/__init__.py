"""MI355X-native Deep Potential (se_e2_a) energy, force and virial.

Submodules:
  synth    seeded synthetic frames and random-initialised parameters (no method arithmetic)
  dpk      ctypes binding of the HIP library libdpk.so (C ABI declared in include/dpk.h)
  torch_op torch.autograd.Function over the device entry point
  build    in-tree build of libdpk.so (hipcc, gfx950)
"""
__all__ = ["synth"]
