"""The paper's comparison solver in FP64 (Sec. 4, "baseline"): a nested
mixed-precision BiCGstab whose single-precision level is preconditioned by
domain decomposition (SAP) with N_SAP = 5.  Test infrastructure only.

The paper names the scheme but not its outer iteration.  Reading adopted:
  * outer level: defect correction with the FP64 operator, r = b - D x, then
    x += e with e an approximate solution of D e = r;
  * inner level: BiCGstab on D e = r, right preconditioned by SAP (N_SAP
    multiplicative red/black sweeps, each domain solved by even-odd minimal
    residual as in the multigrid smoother), stopped at a relative residual
    `inner_tol` or after `inner_max_iters` iterations.
The oracle runs both levels in FP64; the library runs the inner level in FP32.
The paper's domains are 12^4 with SSOR inside; here the domains are the
power-of-two blocks of the field (4^4 in the workloads) with the MR domain
solver of the smoother.
"""
from dataclasses import dataclass

import numpy as np

from .amg import sap


@dataclass
class DDParams:
    sap_sweeps: int = 5           # Sec. 4: N_SAP = 5 for the baseline
    sap_mr_iters: int = 4         # domain solver: fixed MR count, as in the smoother
    inner_tol: float = 1e-4       # relative residual of one inner solve (reading)
    inner_max_iters: int = 500
    max_outer_iters: int = 20


def _dot(a, b):
    return np.vdot(a.ravel(), b.ravel())


def _norm(a):
    return float(np.sqrt(np.real(_dot(a, a))))


def bicgstab(A, M, b, tol, max_iters, x0=None):
    """BiCGstab for A x = b, right preconditioned (A M u = b, x = M u), in the
    standard form of van der Vorst (1992): shadow residual r~ = r0; per step
    p = r + beta (p - omega v), v = A M p, alpha = rho / (r~, v),
    s = r - alpha v, t = A M s, omega = (t, s) / (t, t),
    x += alpha M p + omega M s, r = s - omega t.
    Stops when |r| <= tol |b| (recursive residual).  Returns (x, iterations)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A(x) if x0 is not None else b.copy()
    rt = r.copy()
    nb = _norm(b)
    if nb == 0.0:
        return x, 0
    rho = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    for it in range(1, max_iters + 1):
        if _norm(r) <= tol * nb:
            return x, it - 1
        rho_new = _dot(rt, r)
        beta = (rho_new / rho) * (alpha / omega)
        rho = rho_new
        p = r + beta * (p - omega * v)
        mp = M(p)
        v = A(mp)
        alpha = rho / _dot(rt, v)
        s = r - alpha * v
        ms = M(s)
        t = A(ms)
        tt = np.real(_dot(t, t))
        omega = _dot(t, s) / tt if tt > 0 else 0.0
        x = x + alpha * mp + omega * ms
        r = s - omega * t
    return x, max_iters


def dd_solve(W, b, tol, p=DDParams()):
    """Defect correction around the SAP-preconditioned BiCGstab: returns
    (x, outer iterations, total inner iterations, true relative residual)."""
    nb = _norm(b)
    x = np.zeros_like(b)
    if nb == 0.0:
        return x, 0, 0, 0.0
    M = lambda v: sap(W, v, np.zeros_like(v), p.sap_sweeps, p.sap_mr_iters)   # noqa: E731
    inner = 0
    for outer in range(1, p.max_outer_iters + 1):
        r = b - W.apply(x)
        if _norm(r) <= tol * nb:
            return x, outer - 1, inner, _norm(r) / nb
        e, k = bicgstab(W.apply, M, r, p.inner_tol, p.inner_max_iters)
        inner += k
        x = x + e
    r = b - W.apply(x)
    return x, p.max_outer_iters, inner, _norm(r) / nb
