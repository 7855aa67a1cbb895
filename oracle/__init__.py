"""CPU oracle for the Groth16 matrix-multiplication prover.

TEST INFRASTRUCTURE ONLY: plain, slow, arbitrary-precision Python that states
what the GPU path must compute.  Only tests/, the smoke check and the
benchmark's CPU-baseline leg may import it.  It shares no code with the HIP
library and never imports it.
"""
