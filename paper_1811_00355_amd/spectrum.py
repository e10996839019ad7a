"""Smallest singular value of D on the device, for workload preparation.

sigma_min(D)^2 is the smallest eigenvalue of D^dag D, so it follows from the
largest eigenvalue of (D^dag D)^-1 = D^-1 D^-dag.  By gamma5-hermiticity
(D^dag = g5 D g5, g5 = diag(1, 1, -1, -1) on spin) D^-dag = g5 D^-1 g5, so one
application is two multigrid solves (dd_solve, batched over the block):

    W = g5 D^-1 (g5 X),   Z = D^-1 W = (D^dag D)^-1 X.

Block inverse iteration with Rayleigh-Ritz: X orthonormal (nvec columns),
H = X^dag Z, mu = largest eigenvalue of H, sigma = mu^(-1/2); then X is
re-orthonormalised from Z.  Every estimate is an upper bound on sigma_min that
decreases to it as the block aligns with the lowest singular vectors.

This is a measurement tool around the solver (it chooses masses for the
light-quark workloads); the small dense algebra on the nvec-vector block uses
torch.
"""
import math


def _g5(x):
    """g5 x on canonical [n][V][4][3] vectors stored as [n][12 V]."""
    y = x.view(x.shape[0], -1, 4, 3).clone()
    y[:, :, 2:, :] *= -1
    return y.view(x.shape)


def _orthonormalize(X):
    """Classical Gram-Schmidt, two passes, on the rows of X (complex128)."""
    import torch
    Q = X.clone()
    for i in range(Q.shape[0]):
        for _ in range(2):
            if i:
                c = Q[:i].conj() @ Q[i]
                Q[i] -= c @ Q[:i]
        Q[i] /= torch.linalg.vector_norm(Q[i])
    return Q


def sigma_min(mg, V, nvec=4, iters=8, tol=1e-8, seed=1, rtol=None, log=None):
    """Estimate sigma_min(D) for the operator of multigrid `mg` (lattice of V sites).

    Returns (sigma, history, solve_info): the last estimate, one estimate per
    iteration, and the outer iteration counts of the solves.  Stops early once
    two estimates agree to `rtol` (if given).  Raises if a solve does not
    converge to `tol`."""
    import torch
    n = 12 * V
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    X = torch.complex(torch.randn(nvec, n, generator=gen, device="cuda", dtype=torch.float64),
                      torch.randn(nvec, n, generator=gen, device="cuda", dtype=torch.float64))
    X = _orthonormalize(X)
    hist, its = [], []
    for k in range(iters):
        Y = torch.zeros_like(X)
        info1, _ = mg.dd_solve(nvec, _g5(X), Y, tol)
        W = _g5(Y)
        Z = torch.zeros_like(X)
        info2, _ = mg.dd_solve(nvec, W, Z, tol)
        H = X.conj() @ Z.T
        H = 0.5 * (H + H.conj().T)
        mu = float(torch.linalg.eigvalsh(H).max())
        sigma = 1.0 / math.sqrt(mu)
        hist.append(sigma)
        its.append([i["outer_iters"] for i in info1 + info2])
        if log:
            log(f"[sigma] iteration {k}: sigma_min <= {sigma:.6e} (outer iterations {its[-1]})")
        X = _orthonormalize(Z)
        if rtol is not None and k and abs(hist[-1] - hist[-2]) <= rtol * hist[-1]:
            break
    return hist[-1], hist, its
