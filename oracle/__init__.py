"""Plain FP64 CPU oracle of the thermal PEPS-VMC hot path (arXiv 2409.05285).

This package is test infrastructure.  Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark import it; the product path (the HIP
library and its Python binding) never does, and shares no code with it.

Every function is written for clarity, not speed: NumPy FP64, one chain at a
time, contractions written out as ``einsum`` over named indices, LAPACK (via
NumPy) for QR / SVD / eigh.  Each function cites the passage of the paper it
follows (section, equation, or appendix); where the paper is silent the
docstring states the reading taken.

Modules
-------
lattice      geometry, leg dimensions, parameter / O-row packing
philox       Philox4x64-10 counter-based generator (Salmon et al., SC'11)
network      exact contraction of the single-layer network (no truncation)
bmps         boundary-MPS absorption, compression C_chi, strip contractions
hamiltonian  local energy of the doubled generator, dense operators
ed           exact diagonalisation (sector by sector) and thermal energies
sampler      Metropolis sweep over configurations S = (s, s')
measure      per-sample log|psi|, sign, E_loc and log-derivative row O
sr           sample reductions, SR matvec, conjugate gradient, dense solve
cooling      cooling loop from the beta = 0 identity state
observables  local values of diagonal thermal observables, estimators
simple_update  simple-update Trotter evolution with bond weights
"""
