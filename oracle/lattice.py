"""Lattice geometry: sites, shifts and the domain (aggregate / SAP block) maps.

Sites are lexicographic, site = x + Lx*(y + Ly*(z + Lz*t)).  The lattice is
periodic in x, y, z; a hop that wraps around in t picks up the factor bc_t
(-1: antiperiodic).  Domains are the paper's blocks (Sec. 2 and Sec. 4): the
fine lattice is tiled from the origin by blocks of edge b_mu, each block being
one coarse site (Fig. 1).  The same tiling serves as aggregates of the
interpolation and as SAP domains.  A block is red when the sum of its block
coordinates is even; the coarse parity of a coarse site is its block colour.
"""
import numpy as np


class Lattice:
    def __init__(self, L, block=None, bc_t=-1):
        self.L = tuple(int(l) for l in L)
        self.V = int(np.prod(self.L))
        self.bc_t = bc_t
        # coordinates of every site, each of shape (V,)
        t, z, y, x = np.meshgrid(*[np.arange(self.L[m]) for m in (3, 2, 1, 0)], indexing="ij")
        self.coords = np.stack([x.ravel(), y.ravel(), z.ravel(), t.ravel()])  # [4][V]
        self.parity = self.coords.sum(axis=0) % 2
        self._nbr_cache = {}
        self._all = np.arange(self.V)
        self.block = None
        if block is not None:
            self.set_block(block)

    # -- neighbours -------------------------------------------------------------
    def nbr(self, sites, mu, sign):
        """Neighbour x + sign*mu of each site in `sites`, with its boundary
        factor (bc_t when the hop wraps around in t, else 1)."""
        full = len(sites) == self.V and np.array_equal(sites, self._all)
        key = (mu, sign)
        if full and key in self._nbr_cache:
            return self._nbr_cache[key]
        c = self.coords[:, sites].copy()
        c[mu] += sign
        wrap = (c[mu] < 0) | (c[mu] >= self.L[mu])
        c[mu] %= self.L[mu]
        phase = np.where(wrap & (mu == 3), float(self.bc_t), 1.0)
        res = (self.site_index(c), phase)
        if full:
            self._nbr_cache[key] = res
        return res

    def site_index(self, c):
        x, y, z, t = c
        Lx, Ly, Lz, Lt = self.L
        return x + Lx * (y + Ly * (z + Lz * t))

    # -- blocks / aggregates ----------------------------------------------------
    def set_block(self, block):
        self.block = tuple(int(b) for b in block)
        for mu in range(4):
            if self.L[mu] % self.block[mu]:
                raise ValueError("lattice extent not divisible by the block edge")
        self.NB = tuple(self.L[m] // self.block[m] for m in range(4))
        self.Vc = int(np.prod(self.NB))
        self.Bv = int(np.prod(self.block))
        bc = np.stack([self.coords[m] // self.block[m] for m in range(4)])
        lc = np.stack([self.coords[m] % self.block[m] for m in range(4)])
        NB, b = self.NB, self.block
        # aggregate (coarse site) of each fine site: lexicographic in block coordinates
        self.agg_of_site = bc[0] + NB[0] * (bc[1] + NB[1] * (bc[2] + NB[2] * bc[3]))
        # position of a site inside its block: lexicographic in local coordinates
        self.local_of_site = lc[0] + b[0] * (lc[1] + b[1] * (lc[2] + b[2] * lc[3]))
        # coarse lattice coordinates and colour (= coarse parity) of every block
        ct, cz, cy, cx = np.meshgrid(*[np.arange(NB[m]) for m in (3, 2, 1, 0)], indexing="ij")
        self.coarse_coords = np.stack([cx.ravel(), cy.ravel(), cz.ravel(), ct.ravel()])
        self.color_of_block = self.coarse_coords.sum(axis=0) % 2
        # for each site and direction: does the forward (backward) neighbour stay in the block?
        self.inside_fwd = np.stack([(lc[m] + 1) < b[m] for m in range(4)])
        self.inside_bwd = np.stack([lc[m] > 0 for m in range(4)])
        # sites of each aggregate, ordered by the local index: [Vc][Bv]
        order = np.lexsort((self.local_of_site, self.agg_of_site))
        self.sites_of_agg = order.reshape(self.Vc, self.Bv)

    def coarse_neighbor(self, mu, sign):
        """Index of the coarse neighbour X + sign*mu for every coarse site X (periodic)."""
        c = self.coarse_coords.copy()
        c[mu] = (c[mu] + sign) % self.NB[mu]
        NB = self.NB
        return c[0] + NB[0] * (c[1] + NB[1] * (c[2] + NB[2] * c[3]))
