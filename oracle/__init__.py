"""CPU reference (oracle) for the boxcar single-pulse search of Adamek & Armour (arXiv:1910.08324).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import, call, link or run anything in this package.  The GPU library never does, and this
package never touches the GPU library: the two share no code.  Inputs shared by both sides come
from the `synth` module, which holds none of the search arithmetic.

Contents
  widths       width sets of the exhaustive, BoxDIT and IGRID searches (Sections 3.1, 3.2, Table 1)
  planes       FP64 per-level max-SNR / best-width planes (C, OpenMP) and point evaluations
  brute        direct-sum NumPy evaluation for tiny inputs
  peaks        thresholded 3x3 peak finder (candidate selection) and margin classes for parity
  closed_form  RSNR_max(S), RSNR_min(S) and signal-loss measures of Appendix A and Section 4.2
  loss         pulse-recovery measures (signal loss against the exhaustive search)

Every function is in FP64 and cites the passage it follows.  Parity status of each part is
listed in oracle/PARITY.txt.
"""
