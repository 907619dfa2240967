"""FP64 CPU oracle for the multi-layer collimated-beam UMBIR hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import or run anything in this package; the product path
(the HIP library and its Python binding) never does, and shares no code with it.

Each function is a plain, slow, directly readable statement of what the paper
(Alanazi et al., "Model-Based Reconstruction for Collimated Beam Ultrasound
Systems", ICASSP 2022, arXiv:2202.09703) defines, in float64:

  geometry.py  Snell travel times through planar layers (Sec. 2, Eqs. (4)-(6)),
               apodization (Eq. (12)), transmittance products (Eqs. (3), (7)).
  pulse.py     transmitted pulse, impulse response and its windowed, tabulated
               version (Eqs. (8)-(10)).
  operator.py  the system matrix A applied matrix-free (Eqs. (11), (13)), its
               exact transpose, and the direct-arrival basis D (Eq. (1)).
  prior.py     QGGMRF potential with depth-modulated scale (Eqs. (14)-(17)).
  solver.py    MAP cost (Eqs. (2), (18)), the separable-surrogate update used
               as the parity solver, and ICD (the paper's solver).
  data.py      synthetic measurements y = A x + D g + w (Eq. (1)).

Where the paper is silent or ambiguous the oracle takes one stated reading;
every reading is listed in the design notes and pinned by a test.
"""
from . import geometry, pulse, operator, prior, solver, data  # noqa: F401
