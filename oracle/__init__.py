"""Plain FP64 CPU oracle for the grouped Fourier transform and its solvers.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the HIP library (no kernels, headers,
tables or helpers); only the seeded input generators of ``workloads`` serve both.

What it computes, each function citing the passage it follows:

* ``index_set``  - ANOVA term set U_{d_s} and the grouped frequency index set
  (Sec. 2, eq. pizmosch, eq. metallica, Remark rem:cardinality, eq. groupedset),
  with the coefficient ordering this project fixes where the paper leaves the order of
  the blocks open (Sec. 3, eq. bananarama).
* ``transform``  - the grouped Fourier transform as the direct sum of its definition
  (Definition def:skatoons with eq. somafm), its adjoint (Sec. 3, the stacked adjoint
  after the error remark), the dense d-dimensional Fourier matrix (eq. FM) and the
  analytic node gradient (derivative of the definition; not in the paper).
* ``cosine``     - the grouped transform in the half-period cosine basis on [0, 1]^d
  (Sec. 5 with the extension remark of Sec. 3): index set, forward, adjoint, dense matrix.
* ``lsqr``       - LSQR (Paige & Saunders) for the weighted Tikhonov problem
  (Sec. 4.1, eq. new_min_prob).
* ``fista``      - group-lasso proximal map (Lemma lemma:lennykrawitz, Theorem
  theorem:projection and the root-finding remark after it) and FISTA (Algorithm
  algo:fista, literal backtracking form and the constant-step variant of the remark
  after it), plus a power iteration for the step constant.

Everything is float64 / complex128.  Parity pins: see ``tests/test_oracle_*.py``.
"""
from . import index_set, transform, cosine, lsqr, fista  # noqa: F401
