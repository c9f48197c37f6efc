"""Finite-element pieces of the VTS problem, written out in plain NumPy.

Section 1, problem (1.1): K(rho) = sum_i rho_i K_i, with K_i the element
stiffness K_e scattered to the DOFs of element i.  Section 6.2: trilinear
(Q1) hexahedra for u, one constant density per element, grids obtained by
regular 1->8 refinement of a coarse box of unit cubes.

The element matrix is the isotropic linear-elastic stiffness of a cube of
side h, integrated with the 2x2x2 Gauss rule (exact for Q1 on a cube).  The
paper does not print K_e; the pins are: agreement with exact rational
integration, symmetry, a 6-dimensional rigid-body nullspace.

Local numbering: local node a = ax + 2*ay + 4*az sits at offset (ax, ay, az)
from the element's lowest corner; local DOF = 3*a + component.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

GAUSS_1D = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))
CORNERS = [(a & 1, (a >> 1) & 1, (a >> 2) & 1) for a in range(8)]


def elasticity_matrix(E: float, nu: float) -> np.ndarray:
    """6x6 isotropic D for strains (xx, yy, zz, gamma_xy, gamma_yz, gamma_xz)."""
    c = E / ((1.0 + nu) * (1.0 - 2.0 * nu))
    D = np.zeros((6, 6))
    D[:3, :3] = c * nu
    for i in range(3):
        D[i, i] = c * (1.0 - nu)
        D[3 + i, 3 + i] = c * (1.0 - 2.0 * nu) / 2.0
    return D


def _lagrange(side, t):
    return t if side else 1.0 - t


def _dlagrange(side):
    return 1.0 if side else -1.0


def strain_matrix(t, h: float) -> np.ndarray:
    """6x24 B at reference point t in [0,1]^3 of a cube of side h."""
    B = np.zeros((6, 24))
    for a, (ax, ay, az) in enumerate(CORNERS):
        lx, ly, lz = _lagrange(ax, t[0]), _lagrange(ay, t[1]), _lagrange(az, t[2])
        gx = _dlagrange(ax) * ly * lz / h
        gy = lx * _dlagrange(ay) * lz / h
        gz = lx * ly * _dlagrange(az) / h
        col = 3 * a
        B[0, col + 0] = gx
        B[1, col + 1] = gy
        B[2, col + 2] = gz
        B[3, col + 0], B[3, col + 1] = gy, gx
        B[4, col + 1], B[4, col + 2] = gz, gy
        B[5, col + 0], B[5, col + 2] = gz, gx
    return B


def element_stiffness(E: float = 1.0, nu: float = 0.3, h: float = 1.0) -> np.ndarray:
    """24x24 K_e = int B^T D B dV by the 2x2x2 Gauss rule (weights 1/8 on the
    unit cube, times the volume h^3)."""
    D = elasticity_matrix(E, nu)
    K = np.zeros((24, 24))
    for tx in GAUSS_1D:
        for ty in GAUSS_1D:
            for tz in GAUSS_1D:
                B = strain_matrix((tx, ty, tz), h)
                K += (h ** 3 / 8.0) * B.T @ D @ B
    return K


class Grid:
    """Structured nx x ny x nz grid of cubes with a DOF mask (1 = fixed)."""

    def __init__(self, nx, ny, nz, fixed=None):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.m = self.nx * self.ny * self.nz
        self.n_nodes = (self.nx + 1) * (self.ny + 1) * (self.nz + 1)
        self.n_dof = 3 * self.n_nodes
        if fixed is None:
            fixed = np.zeros(self.n_dof, dtype=np.uint8)
        self.fixed = np.asarray(fixed, dtype=np.uint8)
        self.free = np.nonzero(self.fixed == 0)[0]
        ek, ej, ei = np.meshgrid(np.arange(self.nz), np.arange(self.ny),
                                 np.arange(self.nx), indexing="ij")
        ei, ej, ek = ei.ravel(), ej.ravel(), ek.ravel()
        conn = np.empty((self.m, 8), dtype=np.int64)
        for a, (ax, ay, az) in enumerate(CORNERS):
            conn[:, a] = self.node(ei + ax, ej + ay, ek + az)
        self.conn = conn
        self.dofs = (3 * conn[:, :, None] + np.arange(3)[None, None, :]).reshape(self.m, 24)

    def node(self, i, j, k):
        return i + (self.nx + 1) * (j + (self.ny + 1) * k)

    def node_ijk(self):
        k, j, i = np.meshgrid(np.arange(self.nz + 1), np.arange(self.ny + 1),
                              np.arange(self.nx + 1), indexing="ij")
        return i.ravel(), j.ravel(), k.ravel()

    def mask(self, x):
        y = np.array(x, dtype=np.float64, copy=True)
        y[self.fixed == 1] = 0.0
        return y


def apply_K(grid: Grid, Ke: np.ndarray, rho: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y = K(rho) x on the free DOFs, all-DOF layout (fixed entries of x are
    ignored, fixed entries of y are 0): y = D (sum_i rho_i K_i) D x with D the
    free-DOF mask (problem (1.1), K(rho) = sum rho_i K_i)."""
    xm = grid.mask(x)
    Xe = xm[grid.dofs]                       # m x 24
    Ye = rho[:, None] * (Xe @ Ke.T)
    y = np.bincount(grid.dofs.ravel(), weights=Ye.ravel(), minlength=grid.n_dof)
    y[grid.fixed == 1] = 0.0
    return y


def element_energies(grid: Grid, Ke: np.ndarray, u: np.ndarray) -> np.ndarray:
    """e_i = 1/2 u^T K_i u for every element (Section 2, constraint of (2.1))."""
    Ue = grid.mask(u)[grid.dofs]
    return 0.5 * np.einsum("ei,ij,ej->e", Ue, Ke, Ue)


def element_forces(grid: Grid, Ke: np.ndarray, u: np.ndarray) -> np.ndarray:
    """b_i = K_i u restricted to element i's 24 DOFs (m x 24, not masked)."""
    Ue = grid.mask(u)[grid.dofs]
    return Ue @ Ke.T


def scatter(grid: Grid, Ve: np.ndarray) -> np.ndarray:
    """Assemble per-element 24-vectors into an all-DOF vector, masked."""
    y = np.bincount(grid.dofs.ravel(), weights=np.asarray(Ve).ravel(),
                    minlength=grid.n_dof)
    y[grid.fixed == 1] = 0.0
    return y


def assemble_K(grid: Grid, Ke: np.ndarray, rho: np.ndarray) -> sp.csr_matrix:
    """Assembled K(rho) over ALL DOFs (no mask), CSR."""
    rows = np.repeat(grid.dofs, 24, axis=1).ravel()
    cols = np.tile(grid.dofs, (1, 24)).ravel()
    vals = (rho[:, None, None] * Ke[None, :, :]).ravel()
    return sp.csr_matrix((vals, (rows, cols)), shape=(grid.n_dof, grid.n_dof))


def assemble_K_free(grid: Grid, Ke: np.ndarray, rho: np.ndarray) -> sp.csr_matrix:
    """K(rho) restricted to the free DOFs (the paper's n x n matrix)."""
    K = assemble_K(grid, Ke, rho)
    return K[grid.free][:, grid.free].tocsr()


def element_force_matrix(grid: Grid, be: np.ndarray) -> sp.csc_matrix:
    """B(u) = [K_1 u, ..., K_m u] restricted to free DOFs, n_free x m
    (Section 4 notation B(u); Section 3.2 uses the columns K_i u)."""
    rows = grid.dofs.ravel()
    cols = np.repeat(np.arange(grid.m), 24)
    B = sp.csc_matrix((be.ravel(), (rows, cols)), shape=(grid.n_dof, grid.m))
    return B[grid.free].tocsc()
