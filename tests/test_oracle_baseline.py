"""Pins of the oracle's baseline solver (SAP-preconditioned BiCGstab inside a
defect correction): BiCGstab against a direct solve, its exact two-step
termination on a matrix with two eigenvalues, the outer correction's contraction,
and the whole solve against the dense operator's direct solution."""
import numpy as np

from conftest import rel
from oracle import baseline
import _dense


def test_bicgstab_matches_direct_solve():
    rng = np.random.default_rng(7)
    n = 60
    A = np.eye(n) * 4 + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, it = baseline.bicgstab(lambda v: A @ v, lambda v: v, b, 1e-12, 200)
    assert rel(x, np.linalg.solve(A, b)) < 1e-10 and 0 < it < 60
    # right preconditioning by the exact inverse: one step
    Ai = np.linalg.inv(A)
    x, it = baseline.bicgstab(lambda v: A @ v, lambda v: Ai @ v, b, 1e-12, 10)
    assert rel(x, np.linalg.solve(A, b)) < 1e-10 and it == 1


def test_bicgstab_two_eigenvalues():
    """A diagonalisable matrix with two distinct eigenvalues has a degree-2
    minimal polynomial: BiCGstab (a Krylov method with one polynomial step per
    half iteration) reaches the solution within 2 iterations."""
    rng = np.random.default_rng(8)
    n = 40
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    d = np.where(np.arange(n) < 17, 2.0 + 1j, 5.0 - 0.5j)
    A = Q @ np.diag(d) @ Q.conj().T
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, it = baseline.bicgstab(lambda v: A @ v, lambda v: v, b, 1e-12, 10)
    assert it <= 2 and rel(x, np.linalg.solve(A, b)) < 1e-11


def test_defect_correction_contracts(c1):
    """Each outer step leaves a residual below inner_tol of the previous one."""
    W, b = c1["W"], c1["b"]
    p = baseline.DDParams(inner_tol=1e-2, max_outer_iters=1)
    nb = np.linalg.norm(b)
    prev = None
    x = np.zeros_like(b)
    for k in range(4):
        r = b - W.apply(x)
        cur = np.linalg.norm(r) / nb
        if prev is not None:
            assert cur <= max(1e-2 * prev * 1.0001, 1e-14)
        e, _ = baseline.bicgstab(W.apply, lambda v: v, r, p.inner_tol, p.inner_max_iters)
        x = x + e
        prev = cur
    assert prev < 1e-6


def test_dd_solve_matches_dense_solution(c1):
    """The whole baseline solve on the 4^4 case reaches 1e-10 and agrees with
    the direct solution of the independently built dense D."""
    W, b, U, cfg = c1["W"], c1["b"], c1["U"], c1["cfg"]
    x, outer, inner, res = baseline.dd_solve(W, b, 1e-10)
    D = _dense.dense_D(U, cfg["L"], cfg["m0"], cfg["c_sw"])
    xd = np.linalg.solve(D, _dense.vec(b))
    assert res <= 1e-10 and 1 <= outer <= 5 and inner > 0
    assert rel(_dense.vec(x), xd) < 1e-8
    # SAP(5) as preconditioner cuts the inner iteration count against no preconditioner
    _, k_sap = baseline.bicgstab(W.apply, lambda v: baseline.sap(W, v, np.zeros_like(v), 5, 4), b, 1e-4, 500)
    _, k_none = baseline.bicgstab(W.apply, lambda v: v, b, 1e-4, 500)
    assert k_sap < k_none
