"""Geometric multigrid for the reduced system S of eq. (3.12), Section 6.

Section 6.1: V-cycle correction scheme, Galerkin coarse operators
A_{k-1} = I_k^{k-1} A_k I_{k-1}^k with I_{k-1}^k = (I_k^{k-1})^T, Gauss-Seidel
smoothing.  Section 6.2: regular 1->8 refinement, the standard 27-point
(trilinear) prolongation for u, identity transfer for the extra scalar.

The paper leaves the Gauss-Seidel variant open.  The reading used here (and
by the GPU path): nodal 3x3 block Gauss-Seidel in the multicolour order of
the node parities c = (i&1) + 2(j&1) + 4(k&1); a forward sweep visits colours
0..7 and then the scalar alpha, the backward sweep alpha and then colours
7..0.  One forward sweep before and one backward sweep after the coarse
correction make the V-cycle symmetric, as MINRES needs.  The coarsest level
(the coarse box of the paper's "MG-structured" domain) is solved by a dense
Cholesky factorization.

Everything here is assembled sparse linear algebra on the free DOFs: the
smoother recomputes the full residual r - S z before each colour.

With k load cases (the multi-load extension, `nload` = k) the unknowns are
the stacked free displacements (u_1, ..., u_k) followed by alpha; the
prolongation acts on each load case's block as above, and the smoother's
node block holds the 3k DOFs of a node over all load cases, since the
rank-one element terms of S couple the load cases.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import fe


def coarse_fixed(fine: fe.Grid) -> np.ndarray:
    """A coarse DOF is fixed iff the coincident fine DOF (node (2I,2J,2K)) is."""
    ncx, ncy, ncz = fine.nx // 2, fine.ny // 2, fine.nz // 2
    K, J, I = np.meshgrid(np.arange(ncz + 1), np.arange(ncy + 1),
                          np.arange(ncx + 1), indexing="ij")
    fnode = fine.node(2 * I.ravel(), 2 * J.ravel(), 2 * K.ravel())
    fixed = np.zeros(3 * fnode.size, dtype=np.uint8)
    for c in range(3):
        fixed[c::3] = fine.fixed[3 * fnode + c]
    return fixed


def prolongation_all(coarse: fe.Grid, fine: fe.Grid) -> sp.csr_matrix:
    """Trilinear interpolation over all DOFs: fine node (i,j,k) takes weight
    prod_d w_d from coarse nodes, w = 1 at an even index (coincident node) and
    1/2 from each neighbour at an odd index (27-point scheme)."""
    fi, fj, fk = fine.node_ijk()
    rows, cols, vals = [], [], []

    def opts(t):
        even = (t % 2 == 0)
        a = np.where(even, t // 2, (t - 1) // 2)
        b = np.where(even, t // 2, (t + 1) // 2)
        wa = np.where(even, 1.0, 0.5)
        wb = np.where(even, 0.0, 0.5)
        return [(a, wa), (b, wb)]

    for (ci, wi) in opts(fi):
        for (cj, wj) in opts(fj):
            for (ck, wk) in opts(fk):
                w = wi * wj * wk
                keep = w != 0
                cn = coarse.node(ci, cj, ck)
                fn = np.arange(fine.n_nodes)
                for c in range(3):
                    rows.append(3 * fn[keep] + c)
                    cols.append(3 * cn[keep] + c)
                    vals.append(w[keep])
    P = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(fine.n_dof, coarse.n_dof))
    return P


def check_nested(P_all: sp.csr_matrix, fine: fe.Grid, coarse: fe.Grid) -> bool:
    """True if every fixed fine DOF interpolates from fixed coarse DOFs only
    (then Galerkin on the free DOFs equals masking the all-DOF product)."""
    Pf = P_all[fine.fixed == 1][:, coarse.fixed == 0]
    return Pf.nnz == 0 or np.all(Pf.data == 0)


def node_colors(g: fe.Grid) -> np.ndarray:
    i, j, k = g.node_ijk()
    return (i & 1) + 2 * (j & 1) + 4 * (k & 1)


class Level:
    def __init__(self, grid: fe.Grid, S: sp.csr_matrix, nload: int = 1):
        self.grid = grid
        self.S = S.tocsr()
        self.nload = nload
        self.n = nload * grid.free.size              # u unknowns on this level
        self._blocks()

    def _blocks(self):
        """Per colour: node list, inverse of the free sub-block of S on the
        node's 3 nload DOFs (identity on fixed components), index of each
        component in the stacked free vector (-1 if fixed)."""
        g = self.grid
        nf = g.free.size
        fidx = -np.ones(g.n_dof, dtype=np.int64)
        fidx[g.free] = np.arange(nf)
        col = node_colors(g)
        Sd = self.S
        nb = 3 * self.nload
        self.colors = []
        for c in range(8):
            nodes = np.nonzero(col == c)[0]
            comp1 = fidx[3 * nodes[:, None] + np.arange(3)[None, :]]   # k x 3
            comp = np.concatenate([np.where(comp1 >= 0, comp1 + l * nf, -1)
                                   for l in range(self.nload)], axis=1)
            keep = (comp >= 0).any(axis=1)
            nodes, comp = nodes[keep], comp[keep]
            D = np.zeros((nodes.size, nb, nb))
            for a in range(nb):
                for b in range(nb):
                    ok = (comp[:, a] >= 0) & (comp[:, b] >= 0)
                    ia, ib = comp[ok, a], comp[ok, b]
                    D[ok, a, b] = np.asarray(Sd[ia, ib]).ravel()
                fixed_a = comp[:, a] < 0
                D[fixed_a, a, a] = 1.0
            Dinv = np.linalg.inv(D)
            self.colors.append((comp, Dinv))

    def _color_update(self, c, r, z):
        comp, Dinv = self.colors[c]
        res = r - self.S @ z
        safe = np.where(comp >= 0, comp, 0)
        rn = np.where(comp >= 0, res[safe], 0.0)
        dz = np.einsum("kab,kb->ka", Dinv, rn)
        ok = comp >= 0
        z[comp[ok]] += dz[ok]

    def _alpha_update(self, r, z):
        a = self.n
        row = self.S.getrow(a)
        res_a = r[a] - (row @ z)[0]
        z[a] += res_a / self.S[a, a]

    def gs_forward(self, r, z):
        for c in range(8):
            self._color_update(c, r, z)
        self._alpha_update(r, z)
        return z

    def gs_backward(self, r, z):
        self._alpha_update(r, z)
        for c in reversed(range(8)):
            self._color_update(c, r, z)
        return z


class Hierarchy:
    """Levels k = 1..L (index 0 = coarsest) for S on the grid `fine`, with
    `nload` stacked load cases."""

    def __init__(self, fine: fe.Grid, S: sp.csr_matrix, L: int, nload: int = 1):
        grids = [fine]
        for _ in range(L - 1):
            g = grids[-1]
            if g.nx % 2 or g.ny % 2 or g.nz % 2:
                raise ValueError("grid not divisible for the requested levels")
            grids.append(fe.Grid(g.nx // 2, g.ny // 2, g.nz // 2, coarse_fixed(g)))
        grids = grids[::-1]                           # coarsest first
        self.grids = grids
        self.P = [None]
        for k in range(1, L):
            Pa = prolongation_all(grids[k - 1], grids[k])
            if not check_nested(Pa, grids[k], grids[k - 1]):
                raise ValueError("fixed DOFs are not nested across levels")
            Pf = Pa[grids[k].free][:, grids[k - 1].free]
            self.P.append(sp.block_diag([Pf] * nload + [sp.identity(1)], format="csr"))
        Ss = [None] * L
        Ss[L - 1] = S.tocsr()
        for k in range(L - 1, 0, -1):
            Ss[k - 1] = (self.P[k].T @ Ss[k] @ self.P[k]).tocsr()
        self.levels = [Level(grids[k], Ss[k], nload) for k in range(L)]
        self.chol = sla.cho_factor(Ss[0].toarray(), lower=True)

    def vcycle(self, r, k=None):
        """One V-cycle (correction scheme, zero initial guess)."""
        if k is None:
            k = len(self.levels) - 1
        if k == 0:
            return sla.cho_solve(self.chol, r)
        lev = self.levels[k]
        z = np.zeros_like(r)
        lev.gs_forward(r, z)
        res = r - lev.S @ z
        zc = self.vcycle(self.P[k].T @ res, k - 1)
        z += self.P[k] @ zc
        lev.gs_backward(r, z)
        return z
