"""MACH (randomized Tucker decomposition by sampling) on AMD MI355X.

The compute path lives in libmach.so (hand-written HIP kernels behind the C
ABI of include/mach.h); `paper_0909_4969_amd.mach` is its Python binding and
`paper_0909_4969_amd.serve` the request loop for tensor-stream windows.
Import the submodules explicitly; importing the package itself loads
nothing.
"""
