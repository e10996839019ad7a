"""Euclidean gamma matrices in the chiral representation.

The paper's clover storage (Sec. 3) relies on the chiral representation, in
which the clover term splits into two Hermitian 6x6 blocks.  The matrices
themselves are a choice (the paper prints none):

    gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]   (k = x, y, z)
    gamma_t = [[0, 1], [1, 0]]
    gamma_5 = gamma_x gamma_y gamma_z gamma_t = diag(1, 1, -1, -1)

Direction index mu = 0, 1, 2, 3 <-> x, y, z, t.  A spinor component is
indexed 3*alpha + a (spin alpha, colour a); chirality + is spins 0, 1.
"""
import numpy as np

_s1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_s2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_s3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
_z2 = np.zeros((2, 2), dtype=np.complex128)
_i2 = np.eye(2, dtype=np.complex128)


def _offdiag(a, b):
    return np.block([[_z2, a], [b, _z2]])


GAMMA = np.stack([
    _offdiag(-1j * _s1, 1j * _s1),
    _offdiag(-1j * _s2, 1j * _s2),
    _offdiag(-1j * _s3, 1j * _s3),
    _offdiag(_i2, _i2),
])
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
ID4 = np.eye(4, dtype=np.complex128)
