"""MI355X-native spherical LiDAR surfel rasterizer (Splat-LOAM hot path).

Submodules:
  slr    ctypes binding of libslr.so (render, backward, autograd wrapper)
  synth  seeded synthetic scenes and poses
"""
