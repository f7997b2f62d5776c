"""MI355X-native differentiable one-pixel point rasterizer (ADOP, Sec. 3.1).

Submodules:
  adop      -- ctypes binding of the C-ABI library libadop.so (HIP kernels)
  autograd  -- torch.autograd.Function over the binding
  serve     -- continuous-batching render server
  synth     -- seeded synthetic inputs (no rendering arithmetic)
Importing the package loads nothing native; the binding loads libadop.so on
first use and raises if it is missing.
"""
__version__ = "0.1.0"
