"""Exact stencil coefficients of ENO-MR, derived from their definition.

Test infrastructure: this module belongs to the CPU oracle.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may use it;
the GPU library derives its own tables independently.

Everything here is exact rational arithmetic (``fractions.Fraction``):

* Candidate pool: the 29 linearly stable stencils of the 17-point scheme in the
  order of Eq. (Candidates), Sec. 3.1.  A stencil S_{j-m}^{j+n} is written as the
  pair (m, n).  For a (2r-1)-point scheme of lower order the pool is the same
  list restricted to m <= r-1 and n <= r-1, order kept (the paper lists only the
  17-point pool; this restriction is our reading of "sub-stencils of the global
  stencil S_{j-r+1}^{j+r-1}").

* a_l (Eq. ReconstructedFlux, Tables Flux_reconstruction1/2): the polynomial P of
  degree m+n whose cell averages over I_{j-m}..I_{j+n} equal f_k
  (Eq. Polynomial_Construction) evaluated at x_{j+1/2}.  We solve the moment
  system for P's monomial coefficients exactly and evaluate.

* b_l (Eq. ISCoe, Tables ISCoe1/2): IS = |d^{m+n}P/dx^{m+n}| h^{m+n}
  (Eq. CurrentIS), i.e. (m+n)! times the leading monomial coefficient of P in
  units h = 1.
"""
from fractions import Fraction
from math import factorial

# Eq. (Candidates), Sec. 3.1: S_{j-m}^{j+n} as (m, n), high order to low order.
CANDIDATES_17 = (
    (8, 8), (7, 8), (8, 7), (7, 7), (8, 6), (6, 7), (7, 6), (6, 6), (7, 5),
    (5, 6), (6, 5), (5, 5), (6, 4), (4, 5), (5, 4), (4, 4), (5, 3), (3, 4), (4, 3),
    (3, 3), (2, 3), (3, 2), (2, 2), (1, 2), (2, 1), (1, 1), (0, 1), (1, 0), (0, 0),
)

ORDERS = (5, 7, 9, 11, 13, 15, 17)


def candidates(order):
    """Ordered candidate list for a scheme of odd `order` = 2r-1 in 5..17."""
    if order not in ORDERS:
        raise ValueError("order must be odd in 5..17, got %r" % (order,))
    r = (order + 1) // 2
    return tuple((m, n) for (m, n) in CANDIDATES_17 if m <= r - 1 and n <= r - 1)


def _solve_exact(A, B):
    """Solve A X = B (square A, B a list of columns) by Gauss-Jordan in Fractions."""
    n = len(A)
    M = [list(A[i]) + [B[k][i] for k in range(len(B))] for i in range(n)]
    for col in range(n):
        piv = next(i for i in range(col, n) if M[i][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        p = M[col][col]
        M[col] = [x / p for x in M[col]]
        for i in range(n):
            if i != col and M[i][col] != 0:
                f = M[i][col]
                M[i] = [x - f * y for x, y in zip(M[i], M[col])]
    return [[M[i][n + k] for i in range(n)] for k in range(len(B))]


def _cell_moment(k, d):
    """(1/h) * integral over I_k = [k-1/2, k+1/2] of x^d, with h = 1 and x_j = 0."""
    half = Fraction(1, 2)
    return ((k + half) ** (d + 1) - (k - half) ** (d + 1)) / (d + 1)


def stencil_polynomials(m, n):
    """Monomial coefficients of the cardinal polynomials on S_{j-m}^{j+n}.

    Returns a list over l = -m..n; entry l holds the coefficients c_0..c_{m+n}
    of the degree-(m+n) polynomial whose cell averages are 1 on I_{j+l} and 0 on
    the other cells of the stencil (Eq. Polynomial_Construction with f = e_l).
    """
    deg = m + n
    cells = list(range(-m, n + 1))
    A = [[_cell_moment(k, d) for d in range(deg + 1)] for k in cells]
    rhs = [[Fraction(1 if k == l else 0) for k in cells] for l in cells]
    return _solve_exact(A, rhs)


def a_coefficients(m, n):
    """a_l, l = -m..n, of Eq. (ReconstructedFlux): P(x_{j+1/2}) = sum a_l f_{j+l}."""
    half = Fraction(1, 2)
    return [sum(c * half ** d for d, c in enumerate(poly)) for poly in stencil_polynomials(m, n)]


def b_coefficients(m, n):
    """b_l, l = -m..n, of Eq. (ISCoe): (m+n)! times the leading coefficient of P (h = 1)."""
    deg = m + n
    return [poly[deg] * factorial(deg) for poly in stencil_polynomials(m, n)]


_CACHE = {}


def exact_table(order):
    """[(m, n, a_list, b_list)] for every candidate of `order`, in selection order."""
    if order not in _CACHE:
        _CACHE[order] = [(m, n, a_coefficients(m, n), b_coefficients(m, n))
                         for (m, n) in candidates(order)]
    return _CACHE[order]


def double_table(order):
    """Candidate table with a_l and b_l rounded to the nearest double.

    ``float(Fraction)`` is correctly rounded, so each entry is the double nearest
    to the exact rational.
    """
    return [(m, n, [float(x) for x in a], [float(x) for x in b])
            for (m, n, a, b) in exact_table(order)]
