"""MI355X (gfx950) implementation of the APH digital predistorter of
Li et al., "Parallel Digital Predistortion Design on Mobile GPU and Embedded
Multicore CPU for Mobile Transmitters" (forward apply of Eq. 1 / Algorithm 1,
its adjoint, a batched multi-stream apply and coefficient learning).

Importing the package loads nothing; ``paper_1612_09001_amd.dpd`` loads the
HIP library and fails loudly if it is missing.
"""
__version__ = "0.1.0"
