"""MI355X-native sorted Gaussian-splatting rasterizer (hierarchical per-pixel
resorting on t_opt, as in StopThePop), built as hand-written HIP kernels for
gfx950 behind the C ABI in include/gsr.h.

Submodules:
  gsr    -- ctypes binding of libgsr.so (argument marshalling only)
  synth  -- seeded synthetic scenes and cameras
  build  -- compiles libgsr.so in-tree
"""
