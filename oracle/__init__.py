"""CPU oracles for the GLS solves of Eq. (1): test infrastructure only.

Only the tests, the entry module's smoke check and the benchmark's CPU-baseline
leg import this package; the GPU library never does.  ``GLSOracle`` is the
numpy/LAPACK definition, ``GLSPlain`` the plain single-threaded C one
(``gls_plain.c``), ``GLSWhitenedQR`` the QR route of Section 2.
"""
from .gls import GLSOracle, GLSWhitenedQR, gls_literal, solve_normal_equations, RANK_TOL
from .plain import GLSPlain

__all__ = ["GLSOracle", "GLSPlain", "GLSWhitenedQR", "gls_literal", "solve_normal_equations", "RANK_TOL"]
