"""MI355X (gfx950) implementation of the hot path of image-space collage (arXiv 2406.04008).

Modules:
  scenes   seeded synthetic inputs (outlines, container masks, initial transforms)
  _lib     ctypes declarations of libcollage.so (the C ABI in include/collage.h)
  collage  CollageScene / CollageLoss / CollageGraph: the PyTorch-facing binding
  schedule coarse-to-fine driver (one hipGraph per level)
  autotune tile-size / cache-depth autotuner
"""
__version__ = "0.1.0"
