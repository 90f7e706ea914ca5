"""Staggered-grid finite-difference coefficients, derived exactly.

Test infrastructure (the oracle): only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import anything under
``oracle/``.  The product path shares no code with it.

The paper (Sec. 3.3, "Simulation implementation details") discretises the
stretched pressure-velocity system on a staggered grid with an operator of
order 2M in space and M = 4.  The coefficient values themselves are not printed
(they come from Tan & Huang 2014, which is not available), so the oracle takes
the textbook Taylor construction of a 2M-th order staggered first derivative:

    f'(0) ~ (1/h) * sum_{m=1..M} c_m * ( f((m-1/2)h) - f(-(m-1/2)h) )

is exact for every odd monomial x^(2k-1), k = 1..M, which gives the linear
system  sum_m c_m (2m-1)^(2k-1) = delta_{k,1}.  Even monomials cancel by
symmetry, so the operator is exact for all polynomials of degree <= 2M-1.
The system is solved here in exact rational arithmetic.

Time order (Sec. 3.3 asks for an operator of order 2M in space and fourth
order in time, after Tan & Huang 2014).  With the Taylor coefficients the
leapfrog step is of second order in time.  The time-space-domain staggered
coefficients (Liu & Sen 2011, after Finkelstein & Kastner 2007) instead match
the scheme's own 1D dispersion relation

    sin(w dt / 2) = r * sum_m c_m sin((2m-1) k h / 2),   r = c dt / h,

to the exact w = c k term by term in k h: the powers (kh)^(2k-1),
k = 1..M, agree when  sum_m c_m (2m-1)^(2k-1) = r^(2k-2).  At the reference
speed the 1D step is then of order 2M in space and in time together (the
leading error is (kh)^(2M+1)).  r = 0 gives back the Taylor set.

In 2D and 3D an on-axis stencil cannot reach fourth order in time for oblique
waves: the leapfrog relation sin^2(w dt/2) = r^2 sum_a A_a^2 has mixed terms
(k_a k_b)^2 at fourth order that no sum of squares of on-axis symbols
produces.  Tan & Huang widen each difference by the two-point difference
along its axis in the neighbouring rows of every other axis, with weight b:
A_x = sum_m c_m sin((2m-1) k_x h/2) + 2 b sin(k_x h/2) sum_{o != x} cos(k_o h).
Expanding to fourth order gives b = r^2/24 for the mixed terms, and along each
axis the moments  sum_m c_m (2m-1)^(2k-1) = r^(2k-2) - 2 (d-1) b,  k = 1..M,
in d dimensions.  The divergence takes the same widened stencil, so it stays
the negative transpose of the gradient.
"""
from fractions import Fraction


def _solve_odd_moments(M, rhs):
    """[c_1..c_M] as Fractions solving sum_m c_m (2m-1)^(2k-1) = rhs[k-1]."""
    A = [[Fraction((2 * m - 1) ** (2 * k - 1)) for m in range(1, M + 1)]
         for k in range(1, M + 1)]
    rhs = list(rhs)
    # Gauss-Jordan elimination with exact rationals.
    n = M
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        rhs[col], rhs[piv] = rhs[piv], rhs[col]
        inv = 1 / A[col][col]
        A[col] = [x * inv for x in A[col]]
        rhs[col] = rhs[col] * inv
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col]
                A[r] = [x - f * y for x, y in zip(A[r], A[col])]
                rhs[r] = rhs[r] - f * rhs[col]
    return rhs


def staggered_coefficients_exact(M=4):
    """Return [c_1..c_M] as Fractions solving sum_m c_m (2m-1)^(2k-1) = [k==1]."""
    return _solve_odd_moments(M, [Fraction(1 if k == 1 else 0) for k in range(1, M + 1)])


def staggered_coefficients(M=4):
    """FP64 values of the exact coefficients."""
    return [float(c) for c in staggered_coefficients_exact(M)]


def time_space_coefficients_exact(r, M=4):
    """Time-space-domain coefficients for the Courant number r = c dt / h:
    Fractions solving sum_m c_m (2m-1)^(2k-1) = r^(2k-2), k = 1..M, with r
    taken as the exact rational value of the FP64 number given."""
    rr = Fraction(r) ** 2
    return _solve_odd_moments(M, [rr ** (k - 1) for k in range(1, M + 1)])


def time_space_coefficients(r, M=4):
    """FP64 values of time_space_coefficients_exact(r, M)."""
    return [float(c) for c in time_space_coefficients_exact(r, M)]


def isotropic_time_space_coefficients_exact(r, ndim, M=4):
    """(c_1..c_M, b) as Fractions for the widened stencil in ndim dimensions:
    b = r^2 / 24 and sum_m c_m (2m-1)^(2k-1) = r^(2k-2) - 2 (ndim-1) b."""
    rr = Fraction(r) ** 2
    b = rr / 24
    return _solve_odd_moments(M, [rr ** (k - 1) - 2 * (ndim - 1) * b for k in range(1, M + 1)]), b


def isotropic_time_space_coefficients(r, ndim, M=4):
    """FP64 values of isotropic_time_space_coefficients_exact: ([c_m], b)."""
    c, b = isotropic_time_space_coefficients_exact(r, ndim, M)
    return [float(x) for x in c], float(b)
