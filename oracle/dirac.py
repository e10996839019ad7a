"""Wilson-clover operator, clover term and its packed inverse (FP64).

The operator (standard Sheikholeslami-Wohlert form used by the DD-alpha-AMG
method the paper ports; the paper names the hopping and clover terms in
Sec. 3 but prints no formula):

  (D psi)(x) = A(x) psi(x)
               - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
                              + (1 + gamma_mu) U_mu(x-mu)^dagger psi(x-mu) ]

  A(x) = (4 + m0) 1 - (c_sw / 32) sum_{mu,nu} (gamma_mu gamma_nu) (x) (Q_mu,nu(x) - Q_nu,mu(x))

with Q_mu,nu the sum of the four plaquette leaves in the mu-nu plane that
start and end at x.  Hops that wrap around in t carry the boundary factor;
the clover term uses the raw links.  In the chiral representation A(x) is
block diagonal with two Hermitian 6x6 blocks (chirality + = spins 0,1 and
chirality - = spins 2,3); Sec. 3 stores each block as 6 real diagonal entries
plus 15 complex upper-triangle entries, and stores the full inverse in the
same packed form.  The packing order chosen here: the 6 diagonal reals, then
the upper triangle (r < c) in row-major order.

Spinors are complex128 arrays [V][4][3] (site, spin, colour); links are
[V][4][3][3] (site, mu, row, column).
"""
import numpy as np

from .gamma import GAMMA, ID4

_EYE3 = np.eye(3, dtype=np.complex128)


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


# ---------------------------------------------------------------------------
# clover term
# ---------------------------------------------------------------------------
def leaves(U, lat, sites, mu, nu):
    """Q_mu,nu(x) for x in `sites`: the four plaquettes of the mu-nu plane
    that start and end at x, all with the same orientation."""
    def link(idx, d):
        return U[idx, d]

    def n(idx, d, s):
        return lat.nbr(idx, d, s)[0]

    x = sites
    xpm = n(x, mu, +1)
    xpn = n(x, nu, +1)
    xmm = n(x, mu, -1)
    xmn = n(x, nu, -1)
    xmm_pn = n(xmm, nu, +1)
    xmm_mn = n(xmm, nu, -1)
    xmn_pm = n(xmn, mu, +1)
    Umu, Unu = link(x, mu), link(x, nu)
    l1 = Umu @ link(xpm, nu) @ _dag(link(xpn, mu)) @ _dag(Unu)
    l2 = Unu @ _dag(link(xmm_pn, mu)) @ _dag(link(xmm, nu)) @ link(xmm, mu)
    l3 = _dag(link(xmm, mu)) @ _dag(link(xmm_mn, nu)) @ link(xmm_mn, mu) @ link(xmn, nu)
    l4 = _dag(link(xmn, nu)) @ link(xmn, mu) @ link(xmn_pm, nu) @ _dag(Umu)
    return l1 + l2 + l3 + l4


def clover_matrix(U, lat, m0, c_sw, sites=None):
    """A(x) as dense 12x12 matrices [S][12][12] (index 3*spin + colour)."""
    if sites is None:
        sites = np.arange(lat.V)
    S = len(sites)
    A = np.zeros((S, 12, 12), dtype=np.complex128)
    for a in range(12):
        A[:, a, a] = 4.0 + m0
    if c_sw != 0.0:
        for mu in range(4):
            for nu in range(4):
                if mu == nu:
                    continue
                G = GAMMA[mu] @ GAMMA[nu]
                F = leaves(U, lat, sites, mu, nu) - leaves(U, lat, sites, nu, mu)
                A -= (c_sw / 32.0) * np.einsum("ij,sab->siajb", G, F).reshape(S, 12, 12)
    return A


def chiral_blocks(A):
    """The two 6x6 diagonal blocks [S][2][6][6] of a clover-like matrix."""
    return np.stack([A[:, :6, :6], A[:, 6:, 6:]], axis=1)


def from_chiral_blocks(B):
    S = B.shape[0]
    A = np.zeros((S, 12, 12), dtype=np.complex128)
    A[:, :6, :6] = B[:, 0]
    A[:, 6:, 6:] = B[:, 1]
    return A


_IU = np.triu_indices(6, 1)


def pack_hermitian6(B):
    """[..., 6, 6] Hermitian -> [..., 36] reals: 6 diagonal reals, then the
    15 upper-triangle complex entries (row-major, r < c) as (re, im) pairs."""
    d = np.real(np.diagonal(B, axis1=-2, axis2=-1))
    u = B[..., _IU[0], _IU[1]]
    ri = np.stack([u.real, u.imag], axis=-1).reshape(u.shape[:-1] + (30,))
    return np.concatenate([d, ri], axis=-1)


def unpack_hermitian6(p):
    shp = p.shape[:-1]
    B = np.zeros(shp + (6, 6), dtype=np.complex128)
    for k in range(6):
        B[..., k, k] = p[..., k]
    u = p[..., 6::2] + 1j * p[..., 7::2]
    B[..., _IU[0], _IU[1]] = u
    B[..., _IU[1], _IU[0]] = np.conj(u)
    return B


def clover_inverse_blocks(A):
    """Blockwise inverse of the clover term, [S][2][6][6] (LU with partial
    pivoting through numpy; A is Hermitian but not assumed definite)."""
    return np.linalg.inv(chiral_blocks(A))


# ---------------------------------------------------------------------------
# operator
# ---------------------------------------------------------------------------
def apply_blockdiag(B, psi):
    """Apply per-site chirality blocks B [V][2][6][6] to psi [V][4][3]."""
    v = psi.reshape(-1, 2, 6, 1)
    return (B @ v).reshape(psi.shape)


def apply_clover(A, psi):
    """A(x) psi(x) with A given as dense [V][12][12]."""
    return (A @ psi.reshape(-1, 12, 1)).reshape(psi.shape)


def hop_one(U, lat, psi, mu, sign, sites=None):
    """One hop of the hopping term at `sites` (default all):
    sign = +1:  -1/2 (1 - gamma_mu) U_mu(x) psi(x+mu)
    sign = -1:  -1/2 (1 + gamma_mu) U_mu(x-mu)^dagger psi(x-mu)"""
    if sites is None:
        sites = np.arange(lat.V)
    y, ph = lat.nbr(sites, mu, sign)
    if sign > 0:
        spin = (ID4 - GAMMA[mu]) @ psi[y]                  # spin matrix on the spin index
        t = spin @ np.swapaxes(U[sites, mu], -1, -2)       # t[s,i,a] = sum_b U[a,b] spin[i,b]
    else:
        spin = (ID4 + GAMMA[mu]) @ psi[y]
        t = spin @ np.conj(U[y, mu])                       # t[s,i,a] = sum_b conj(U[b,a]) spin[i,b]
    return -0.5 * t * ph[:, None, None]


def hop_terms(U, lat, psi, mask_fwd=None, mask_bwd=None, sites=None):
    """-1/2 sum_mu [(1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^dag psi(x-mu)]
    at `sites` (default all).  Optional boolean masks [4][V] keep only the hops
    for which they are true (Dirichlet block restriction)."""
    if sites is None:
        sites = np.arange(lat.V)
    out = np.zeros((len(sites), 4, 3), dtype=np.complex128)
    for mu in range(4):
        tf = hop_one(U, lat, psi, mu, +1, sites)
        tb = hop_one(U, lat, psi, mu, -1, sites)
        if mask_fwd is not None:
            tf *= mask_fwd[mu][sites][:, None, None]
            tb *= mask_bwd[mu][sites][:, None, None]
        out += tf + tb
    return out


def apply_D(U, A, lat, psi, sites=None):
    """(D psi) at `sites` (default all) for one fine vector psi [V][4][3]."""
    if sites is None:
        return apply_clover(A, psi) + hop_terms(U, lat, psi)
    return apply_clover(A[sites], psi[sites]) + hop_terms(U, lat, psi, sites=sites)


class WilsonClover:
    """The fine operator for one gauge field: links, clover, clover inverse."""

    def __init__(self, U, lat, m0, c_sw, A=None):
        """`A` overrides the clover term computed from the links (used to run
        the operator on stored, rounded operands)."""
        self.U = U
        self.lat = lat
        self.m0 = m0
        self.c_sw = c_sw
        self.A = clover_matrix(U, lat, m0, c_sw) if A is None else A
        self.Ainv_blocks = clover_inverse_blocks(self.A)

    def apply(self, psi):
        return apply_D(self.U, self.A, self.lat, psi)

    def apply_dagger(self, psi):
        """D^dagger = gamma5 D gamma5 (used only by tests and the mass tuning)."""
        g5 = np.array([1, 1, -1, -1])[None, :, None]
        return g5 * self.apply(g5 * psi)

    # -- block (Dirichlet) pieces used by SAP ------------------------------------
    def hop_block(self, psi):
        """Hopping term restricted to every block: hops leaving a block dropped."""
        return hop_terms(self.U, self.lat, psi, self.lat.inside_fwd, self.lat.inside_bwd)

    def apply_block(self, psi):
        """D_B psi for all blocks at once (block diagonal, Dirichlet boundaries)."""
        return apply_clover(self.A, psi) + self.hop_block(psi)

    def apply_Ainv(self, psi):
        return apply_blockdiag(self.Ainv_blocks, psi)
