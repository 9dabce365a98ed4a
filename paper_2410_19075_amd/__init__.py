"""MI355X-native hot path for the network-dynamics method of arXiv 2410.19075.

Submodules:
  nd      ctypes binding of the C-ABI library libnd.so (include/nd.h)
  inputs  seeded synthetic inputs (SplitMix64), shared with the tests
  build   hipcc build of libnd.so for gfx950
"""
