"""Exact one-dimensional Bernstein tables for the oracle.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
module; it is used by ``tests/``, the smoke check and the CPU-baseline leg of
the benchmark.

Source: Kuzmin, Hajduk & Vedral, "An element-based convex limiting framework
for continuous Galerkin methods with nonlinear stabilization",
arXiv:2509.04673 (cited below as [KHV]).  Equation numbers follow the order
of the arXiv source.

[KHV §2.1] uses the Bernstein basis: nonnegative functions forming a
partition of unity.  On the reference interval [0, 1] the degree-p basis is
    B_a(t) = C(p, a) t^a (1 - t)^(p - a),   a = 0..p.
Every integral below is computed in exact rational arithmetic from the
monomial expansion of these polynomials and only then rounded to float64.
"""
from fractions import Fraction
from functools import lru_cache
from math import comb, factorial

import numpy as np


# ---------------------------------------------------------------------------
# exact polynomial helpers (monomial coefficients, lowest degree first)
# ---------------------------------------------------------------------------
def _mul(a, b):
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def _der(a):
    return [a[k] * k for k in range(1, len(a))] or [Fraction(0)]


def _int01(a):
    return sum(c / (k + 1) for k, c in enumerate(a))


def _eval(a, t):
    """Evaluate a monomial-coefficient polynomial at float points t."""
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros_like(t)
    for c in reversed(a):
        out = out * t + float(c)
    return out


@lru_cache(maxsize=None)
def basis_poly(p, a):
    """Monomial coefficients of B_a^p(t) = C(p,a) t^a (1-t)^(p-a)."""
    coeffs = [Fraction(0)] * (p + 1)
    for j in range(p - a + 1):
        coeffs[a + j] += Fraction(comb(p, a) * comb(p - a, j) * (-1) ** j)
    return tuple(coeffs)


def _table(p, fa, fb):
    return [[_int01(_mul(fa(basis_poly(p, a)), fb(basis_poly(p, b))))
             for b in range(p + 1)] for a in range(p + 1)]


def _ident(x):
    return list(x)


@lru_cache(maxsize=None)
def exact_tables(p):
    """Exact rational reference-interval integrals for degree p.

    mass[a][b]  = int_0^1 B_a B_b
    cdiv[a][b]  = int_0^1 B_a B_b'      (test function a, derivative on b)
    cgrad[a][b] = int_0^1 B_a' B_b      (derivative on the test function)
    stiff[a][b] = int_0^1 B_a' B_b'
    lump[a]     = int_0^1 B_a
    """
    return dict(
        mass=_table(p, _ident, _ident),
        cdiv=_table(p, _ident, _der),
        cgrad=_table(p, _der, _ident),
        stiff=_table(p, _der, _der),
        lump=[_int01(list(basis_poly(p, a))) for a in range(p + 1)],
    )


def tables(p):
    """Float64 versions of :func:`exact_tables` as numpy arrays."""
    ex = exact_tables(p)
    return {k: np.array([[float(x) for x in row] for row in v])
            if isinstance(v[0], list) else np.array([float(x) for x in v])
            for k, v in ex.items()}


def gauss(n):
    """n-point Gauss-Legendre rule mapped to [0, 1] (library routine)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def basis_values(p, t):
    """Matrix V[q, a] = B_a^p(t_q) at float points t (any real t)."""
    return np.stack([_eval(basis_poly(p, a), t) for a in range(p + 1)], axis=-1)


def basis_derivs(p, t):
    """Matrix V[q, a] = (B_a^p)'(t_q)."""
    return np.stack([_eval(_der(list(basis_poly(p, a))), t)
                     for a in range(p + 1)], axis=-1)


def derivative_factor(p, k):
    """p! / (p-k)!: the factor of the k-th derivative of a degree-p Bernstein
    polynomial written with k-th forward differences of its coefficients,
        d^k/dt^k sum_a c_a B_a^p = p!/(p-k)! sum_a (Delta^k c)_a B_a^{p-k}
    (textbook identity; it makes the derivative of a constant exactly zero).
    """
    return factorial(p) // factorial(p - k)
