"""FP64 CPU oracle for the ChFSI hot path -- TEST INFRASTRUCTURE ONLY.

This package is the independent reference that the HIP path is checked
against.  It is imported only by the tests, by the smoke check and by the
benchmark's CPU-baseline leg; the product path (the C-ABI library and its
Python binding) never imports, calls or links it.  It shares no code with the
HIP path: quadrature rules, basis tables, mesh numbering, cell matrices,
projectors, the assembled operator and every eigensolver step are written here
from the paper's equations, in plain numpy/scipy, in float64/complex128.

Modules
  fe          GLL/GL rules, Lagrange tables, periodic hexahedral mesh, lumped mass
  projectors  real-harmonic Gaussian projectors, angular-momentum matrices, Delta
  hamiltonian assembled sparse H^k and M^{-1/2} H^k M^{-1/2}
  chfsi       Lanczos bound, scaled Chebyshev filter, CholGS, Rayleigh-Ritz, passes
  adjoint     density / magnetisation closed forms for the filter adjoint

Parity status: every function is pinned by a closed form, an invariant or a
brute-force check in tests/test_oracle_*.py except where its docstring says
"parity unpinned".
"""
