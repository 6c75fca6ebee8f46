"""FP64 CPU oracle of the MIPWA likelihood (test infrastructure only).

This package is the plain, slow, obviously-correct reference that the GPU library is checked
against.  Only the tests, the smoke check and the benchmark's CPU-baseline leg may import it; the
product library never calls it and shares no code with it.

What it computes follows the paper "Model-independent partial wave analysis using a
massively-parallel fitting framework" (Sun, Aoude, dos Reis, Sokoloff):

* Sec. 2, Eq. 1 -- the coherent amplitude sum A(s12, s13) = sum_L sum_k c_k^L A_k^L, truncated at L = 2;
* Sec. 2 -- P/D waves as relativistic Breit-Wigners times a real spin-dependent angular factor;
* Sec. 2 -- the MIPWA S-wave: N knots spanning the m^2(h+h-) spectrum, A_0(s_k) = a_k exp(i phi_k),
  cubic-spline interpolation in the complex plane between knots;
* Sec. 4 -- Bose symmetrisation over the two m^2(h+h-) axes;
* Sec. 2 and Sec. 4 -- the unbinned maximum-likelihood fit with the normalisation integral
  recomputed every iteration from points spread over the Dalitz plane;
* Sec. 2 -- the isobar S-wave (a constant non-resonant term plus scalar Breit-Wigners) and, as the
  abstract's source text names it, the knots as real and imaginary parts (module forms).

The paper leaves the spline boundary conditions, the Breit-Wigner form, barrier factors and angular
terms to references it does not reproduce.  The readings used here (natural spline on Re and Im,
PDG/CLEO mass-dependent width with Blatt-Weisskopf factors and Zemach tensors, no 1/sqrt(2) in the
symmetrisation) are the same in every module; each function names the reading it takes.

Parity status: every function here is pinned by tests in tests/test_oracle_*.py against closed
forms, library special cases, brute force or invariants.  Absolute agreement with the paper's own
fitted values cannot be checked (the paper prints none), so that comparison is parity unpinned.
"""
from .model import Model, Res  # noqa: F401
from . import kinematics, spline, resonance, likelihood, fit, philox, generate, forms  # noqa: F401
