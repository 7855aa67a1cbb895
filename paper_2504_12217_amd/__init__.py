"""MI355X Groth16 prover for the matrix-multiplication statement Y = X W.

The prover is libzkvc.so (hand-written HIP kernels for gfx950 behind a C
ABI, include/zkvc.h); `zkvc` is its ctypes binding.  Build with
`python -m paper_2504_12217_amd.build`.
"""
