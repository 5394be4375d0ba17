"""CPU oracle for the GLS solves of Eq. (1): test infrastructure only.

Only the tests, the entry module's smoke check and the benchmark's CPU-baseline
leg import this package; the GPU library never does.
"""
from .gls import GLSOracle, GLSWhitenedQR, gls_literal, solve_normal_equations, RANK_TOL

__all__ = ["GLSOracle", "GLSWhitenedQR", "gls_literal", "solve_normal_equations", "RANK_TOL"]
