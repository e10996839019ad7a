"""Seeded generators for synthetic lattice inputs.

Canonical layouts (shared by the oracle and the library's pack/unpack):
  * gauge links  : complex128 [V][4][3][3]   (site, direction mu = x,y,z,t, row, column)
  * fine vectors : complex128 [nrhs][V][4][3] (rhs, site, spin, colour)
  * site index   : x + Lx*(y + Ly*(z + Lz*t))

The workload recipe follows the paper's test setting only in shape: a
synthetic, seeded SU(3) field stands in for the missing production gauge
configuration.  Links are U = exp(i*eps*H) with H traceless Hermitian built
from complex Gaussian entries, then reunitarised row by row.
"""
import numpy as np
import torch


def lattice_volume(L):
    v = 1
    for l in L:
        v *= int(l)
    return v


def _rng(seed):
    return np.random.Generator(np.random.Philox(key=int(seed)))


def _herm_traceless(A):
    H = 0.5 * (A + np.conj(np.swapaxes(A, -1, -2)))
    tr = np.trace(H, axis1=-2, axis2=-1).real / 3.0
    for a in range(3):
        H[..., a, a] -= tr
    return H


def _expm_i(H, eps, squarings=4, degree=12):
    """exp(i*eps*H) for a stack of 3x3 matrices: scaling and squaring with a
    truncated Taylor series (|eps*H| / 2**squarings < 0.3, so the truncation
    error is below 1e-17).  The batched 3x3 products use torch's threaded CPU
    matmul purely for speed."""
    X = torch.from_numpy((1j * eps / (2.0 ** squarings)) * H)
    eye = torch.eye(3, dtype=torch.complex128).expand(X.shape[0], 3, 3)
    # Horner: I + X(I + X/2(I + X/3(...)))
    E = eye.clone()
    for k in range(degree, 0, -1):
        E = eye + torch.matmul(X, E) / k
    for _ in range(squarings):
        E = torch.matmul(E, E)
    return E.numpy()


def _reunitarise(U):
    r0 = U[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = U[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def su3_random(count, eps, seed, chunk=1 << 20):
    """`count` SU(3) matrices exp(i*eps*H), H traceless Hermitian with
    complex Gaussian entries (real and imaginary parts N(0,1)), drawn in
    order from a Philox stream keyed by `seed`."""
    g = _rng(seed).standard_normal(size=(count, 3, 3, 2))
    out = np.empty((count, 3, 3), dtype=np.complex128)
    for s in range(0, count, chunk):
        e = min(count, s + chunk)
        A = g[s:e, ..., 0] + 1j * g[s:e, ..., 1]
        U = _expm_i(_herm_traceless(A), eps)
        out[s:e] = _reunitarise(U)
    return out


def su3_field(L, eps, seed):
    """Gauge field, complex128 [V][4][3][3]."""
    V = lattice_volume(L)
    return su3_random(V * 4, eps, seed).reshape(V, 4, 3, 3)


def gauss_spinor(L, nrhs, seed):
    """Complex Gaussian fine vectors, complex128 [nrhs][V][4][3]."""
    V = lattice_volume(L)
    g = _rng(seed).standard_normal(size=(nrhs, V, 4, 3, 2))
    return g[..., 0] + 1j * g[..., 1]


def gauss_vectors(n, V, seed, ncomp=12):
    """n complex Gaussian vectors of V*ncomp entries: complex128 [n][V][ncomp]."""
    g = _rng(seed).standard_normal(size=(n, V, ncomp, 2))
    return g[..., 0] + 1j * g[..., 1]


def point_sources(L, site=0):
    """The 12 spin-colour point sources at one site: b_(alpha,a)(x) =
    delta(x, site) delta(spin, alpha) delta(colour, a);  [12][V][4][3]."""
    V = lattice_volume(L)
    b = np.zeros((12, V, 4, 3), dtype=np.complex128)
    for k in range(12):
        b[k, site, k // 3, k % 3] = 1.0
    return b
