"""Plain float64 CPU oracle for the limited CG-WENO SSP-RK stage.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this
package.  The HIP library never links, loads or calls it, and the two share
no code: this package builds its own exact rational Bernstein tables, dense
element matrices and dense LU factorisations and follows the paper's
formulas literally.

Method: Kuzmin, Hajduk & Vedral, "An element-based convex limiting framework
for continuous Galerkin methods with nonlinear stabilization",
arXiv:2509.04673 ([KHV]).  Equation numbers follow the arXiv source.

Parity status per function (pins live in tests/test_oracle_*.py):
  bernstein tables        pinned (closed forms, partition of unity)
  consistent mass solve   pinned (dense global assembly on tiny meshes)
  projected gradient      pinned (exact on global polynomials)
  WENO sensor             pinned (semi-norm closed forms, gamma = 1 on global
                          polynomials, range, affine invariance); the choice
                          of candidate polynomials itself is a reading
  residual / udot         pinned (exact advection of polynomials, zero sum)
  facet fluxes, dt_e      pinned (closed form dt_e, 1D hand-derived LO step)
  flux limiter            pinned (maximality by brute force)
  slope limiter           pinned (maximality by brute force)
  Appendix A limiter      pinned (admissibility on an alpha grid)
  stage / SSP-RK3         pinned (equivalence theorem, conservation,
                          constant states, IDP, design order)
  non-periodic 1D line    pinned (Galerkin exactness on polynomials with
  (b_i, f^partial, g_i^e) consistent inflow data, the weak form with test
                          function 1, upwind P1 low-order step with an
                          inflow state, equivalence theorem, walls carry
                          no mass or energy, interior = periodic scheme)
"""
from .mesh import Mesh, multi_indices            # noqa: F401
from .scheme import Oracle, Params, Problem, CFLViolation   # noqa: F401
