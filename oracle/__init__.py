"""FP64 CPU oracle for the Hadamard-Babich (HB) volume integrator.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check of the
package's entry script and the CPU-baseline leg of the benchmark may import
this package.  The product path (the HIP library and its Python binding)
never calls it, and it shares no code with that path: it reads the same
seeded inputs (``hb_inputs``) and nothing else.

What it computes is the plain definition of the discretised integrator,
U = K (h^d s) (Sec. 3.1, eq. m_v2v), with
  * K_ij = v0 f_{-(d-2)/2}(omega, tau) + v1 f_{1-(d-2)/2}(omega, tau) for
    i != j (eq. babich with N = 1, terms from eq. termf),
  * tau^2, v0, v1 from the Chebyshev interpolation of the tables
    (eq. chebinterp in its blocked form eq. chebinterpblock),
  * K_ii = h^-d times the integral of the leading HB term over cell i
    (Appendix A: lemma eq. HankelIntegral2dlemma in 2D, Q_s of eq. e312 in
    3D).
Every function is dense and O(N_v) per output row; nothing is compressed.
``oracle.inclusion`` adds the curve inclusion of eq. m_v2v_inclu.
"""
from .hb_oracle import (cheb_nodes, lagrange_1d, interp_weights, interpolate,
                        hb_terms, self_term, entries, apply, apply_adjoint,
                        dense)
from . import inclusion

__all__ = ["cheb_nodes", "lagrange_1d", "interp_weights", "interpolate",
           "hb_terms", "self_term", "entries", "apply", "apply_adjoint",
           "dense", "inclusion"]
