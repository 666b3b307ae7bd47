"""Uniform box meshes of Bernstein Q_p elements for the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

[KHV §2.1, Table 1] index sets: N_e (nodes of element e), E_i (elements
containing node i), B_e (facet neighbours of e).  On a periodic box of n_k
cube cells of side h along axis k with degree p there are L_k = p n_k unique
nodes per axis; node (i_1..i_d) has global index sum_k i_k S_k with x
fastest, element (e_1..e_d) owns local nodes a in [0, p]^d at global
positions (p e_k + a_k) mod L_k.  Local node numbering is lexicographic with
the first axis fastest.

A non-periodic mesh (``periodic=False``) is a 1D line [lo, hi] of n cells:
L = p n + 1 nodes, element e owns nodes p e .. p e + p, and the two end
facets are boundary facets (index e' > E_h of [KHV Table 1]): element 0 has
no low neighbour and element n - 1 no high one (``neighbour`` returns -1).
"""
from dataclasses import dataclass
from itertools import product

import numpy as np


@dataclass
class Mesh:
    d: int
    p: int
    n: tuple          # elements per axis
    lo: tuple
    hi: tuple
    periodic: bool = True

    def __post_init__(self):
        self.n = tuple(int(x) for x in self.n)
        assert len(self.n) == self.d and 1 <= self.d <= 3
        assert self.periodic or self.d == 1, "non-periodic meshes are 1D lines"
        hs = [(self.hi[k] - self.lo[k]) / self.n[k] for k in range(self.d)]
        assert max(hs) - min(hs) <= 1e-12 * max(hs), "cube cells required"
        self.h = hs[0]
        extra = 0 if self.periodic else 1
        self.L = tuple(self.p * nk + extra for nk in self.n)
        self.N = int(np.prod(self.L))
        self.E = int(np.prod(self.n))
        self.nloc = (self.p + 1) ** self.d
        self.node_stride = tuple(int(np.prod(self.L[:k])) for k in range(self.d))
        self.elem_stride = tuple(int(np.prod(self.n[:k])) for k in range(self.d))

    # -- element multi-indices and connectivity ----------------------------
    def element_index(self):
        """(E, d) integer multi-indices of all elements, id order."""
        grids = np.meshgrid(*[np.arange(nk) for nk in self.n], indexing="ij")
        # element id = sum e_k T_k with axis 0 fastest
        idx = np.stack([g.ravel() for g in grids], axis=1)
        ids = idx @ np.array(self.elem_stride)
        out = np.empty_like(idx)
        out[ids] = idx
        return out

    def local_index(self):
        """(nloc, d) local multi-indices a, local id order (axis 0 fastest)."""
        out = np.empty((self.nloc, self.d), dtype=np.int64)
        for loc in range(self.nloc):
            r = loc
            for k in range(self.d):
                out[loc, k] = r % (self.p + 1)
                r //= self.p + 1
        return out

    def connectivity(self):
        """conn[e, loc] = global node index of local node loc of element e."""
        eidx = self.element_index()
        aidx = self.local_index()
        g = np.zeros((self.E, self.nloc), dtype=np.int64)
        for k in range(self.d):
            pos = (self.p * eidx[:, k][:, None] + aidx[:, k][None, :]) % self.L[k]
            g += pos * self.node_stride[k]
        return g

    def neighbour(self, axis, side):
        """Element id of the facet neighbour of every element along `axis`
        on the low (side = -1) or high (side = +1) side: periodic, or -1
        across a boundary facet of a non-periodic line."""
        eidx = self.element_index().copy()
        if not self.periodic:
            nb = eidx[:, axis] + side
            return np.where((nb >= 0) & (nb < self.n[axis]), nb, -1)
        eidx[:, axis] = (eidx[:, axis] + side) % self.n[axis]
        return eidx @ np.array(self.elem_stride)

    def node_coords(self):
        """(N, d) coordinates of the Bernstein nodal points x_j, used only to
        initialise u_j(0) = u_0(x_j) [KHV §5]."""
        grids = np.meshgrid(*[np.arange(Lk) for Lk in self.L], indexing="ij")
        idx = np.stack([g.ravel() for g in grids], axis=1)
        ids = idx @ np.array(self.node_stride)
        out = np.empty(idx.shape, dtype=np.float64)
        out[ids] = np.array(self.lo) + self.h * idx / self.p
        return out

    def facet_local_nodes(self, axis, side):
        """Local ids of the nodes on the low (a_axis = 0) or high (a_axis = p)
        facet, in lexicographic order of the remaining axes."""
        a = self.local_index()
        target = 0 if side < 0 else self.p
        return np.nonzero(a[:, axis] == target)[0]

    def multiplicity(self):
        """|E_i| for every node: number of elements containing node i."""
        cnt = np.zeros(self.N, dtype=np.int64)
        np.add.at(cnt, self.connectivity().ravel(), 1)
        return cnt


def multi_indices(d, p):
    """All derivative multi-indices k with 1 <= |k| <= p ([KHV eq. (8)])."""
    return [k for k in product(range(p + 1), repeat=d) if 1 <= sum(k) <= p]
