"""FP64 CPU oracle for the Newton-Stokes operator -- TEST INFRASTRUCTURE ONLY.

This package is the slow, plain reference that the GPU engine is checked
against.  Only the test-suite, the smoke check in ``__graft_entry__`` and the
CPU-baseline leg of ``bench.py`` may import it; the engine itself never does,
and it shares no code, tables or helpers with the engine.

What it computes, by definition (no sum factorisation, no blocking):

* reference tables: tensor Gauss-Lobatto Lagrange basis on Gauss points,
  the mapped P_{k-1} and the Gauss-point Q_{k-2} pressure bases
  (Sec. 3.2.1-3.2.2, Sec. 6);
* element restrictions R_e by point location in a coarse neighbour and
  evaluation of its Lagrange basis (Sec. 3.2.1, figure "hanging"), with
  periodic lateral axes matched modulo the period (Sec. 4.3);
* dense element residuals and Jacobians by full tensor quadrature of
  eq. (weak) and eq. (newton) with the tensor of eq. (rank4), or the
  Picard operator (Sec. 2.2-2.3);
* the basal Robin term and u.n = 0 by a component mask or by nodal frames
  (eq. (robin), eq. (weak));
* global assembly A = sum_e R_e^T A_e R_e (Sec. 3.2.1) with scipy.sparse;
* the residual VJP and the energy functional of the appendix;
* the low-order approximation F~ of the velocity block on the Gauss-Lobatto
  sub-grid (Sec. 5): trilinear sub-cells, 2-point Gauss-Lobatto quadrature,
  nodal coefficients from the high-order state, assembled with R_e;
* a solved state by Newton's method with direct sparse solves, and the adjoint
  gradient of a functional of the solved state with respect to logA and beta
  (Sec. 2.3), by a direct solve with the transposed Jacobian.

Every function carries "parity unpinned" in its docstring where no
independent pin exists; the pins live in ``tests/test_oracle_*.py``.
"""
from .reference import ReferenceElement
from .restriction import build_restriction
from .stokes import StokesOracle
from .adjoint import adjoint_gradient, newton_solve
from .loworder import low_order_matrix

__all__ = ["ReferenceElement", "build_restriction", "StokesOracle", "adjoint_gradient", "newton_solve",
           "low_order_matrix"]
