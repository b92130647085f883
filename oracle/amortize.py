"""Break-even call count (Equation 2; test infrastructure).

With a one-off planning cost of P plain-CSR SpMV times and a tuned SpMV that
is S times faster than plain CSR, n calls pay off when
P * t_CSR + n * t_CSR / S < n * t_CSR, i.e. n > P * S / (S - 1).  The paper's
numbers (P = 19, S = 3) give n > 28.5, hence at least 29 calls.  (Read
literally, the printed left side multiplies n/3 by the tuned time instead of
the CSR time, which would give n > 21.4 and contradicts the stated 29; the
reading above is the one that reproduces the paper's own result.)
"""
import math


def break_even_calls(plan_cost_in_csr: float, speedup: float) -> float:
    """Smallest real n with plan + n/speedup < n (in plain-CSR SpMV units)."""
    if speedup <= 1.0:
        return math.inf
    return plan_cost_in_csr * speedup / (speedup - 1.0)


def min_calls(plan_cost_in_csr: float, speedup: float) -> int:
    n = break_even_calls(plan_cost_in_csr, speedup)
    return math.inf if n == math.inf else math.floor(n) + 1
