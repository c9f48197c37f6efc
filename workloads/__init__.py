"""Seeded synthetic inputs for the 3D variable-thickness-sheet (VTS) problem.

This module only *describes* problems: the hexahedral grid, which degrees of
freedom are held fixed, the nodal load vector, the volume bound V and the
density bounds.  It holds none of the method's arithmetic (no stiffness, no
penalty function, no solver), so both the CPU oracle and the GPU path may use
it without sharing any of the method.

Geometry follows the "MG-structured cuboid" of Section 7 (Numerical
experiments): a coarse mx x my x mz mesh of unit cubes refined l-1 times, so
the finest grid has nx = mx * 2**(l-1) elements along x, etc.  Nodes are
numbered lexicographically with x fastest, node(i, j, k) = i + (nx+1)*(j +
(ny+1)*k); displacement DOF c (0=x, 1=y, 2=z) of node p is 3*p + c.
Elements are numbered the same way over (nx, ny, nz).

Boundary conditions (Section 7, the cantilever and bridge descriptions):
  * cantilever: every node of the face x = 0 is fixed in all directions;
  * bridge: the four corner nodes of the bottom face z = 0 are fixed in all
    directions.
The load magnitudes and patch shapes are not given in the paper; the
readings used here: unit nodal loads on the cantilever edge, a unit pressure
on the whole bridge top face (consistent bilinear nodal forces), and seeded
unit point loads for the three-load cantilever.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = [
    "Problem", "cantilever_edge", "bar_rollers", "cantilever_points", "bridge_top",
    "paper_cantilever", "paper_bridge", "mg_levels", "config",
    "random_rho", "random_vector", "serving_requests", "CONFIGS",
    "load_cases", "with_load_cases", "cantilever_two_loads", "multi_config", "point_cases",
]


@dataclass
class Problem:
    """A VTS instance on an nx x ny x nz grid of cubic hexahedra of side h."""
    name: str
    nx: int
    ny: int
    nz: int
    levels: int
    fixed: np.ndarray          # uint8, 3*(nx+1)(ny+1)(nz+1); 1 = fixed DOF
    f: np.ndarray              # float64, same length; zero at fixed DOFs
    V: float                   # volume bound, sum(rho) = V
    rho_lo: float = 1e-3
    rho_hi: float = 1.0
    E: float = 1.0
    nu: float = 0.3
    h: float = 1.0
    extra: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_nodes(self) -> int:
        return (self.nx + 1) * (self.ny + 1) * (self.nz + 1)

    @property
    def n_dof(self) -> int:
        return 3 * self.n_nodes

    @property
    def n(self) -> int:
        """Number of free displacement DOFs (the paper's n)."""
        return int(self.n_dof - int(self.fixed.sum()))

    def node(self, i, j, k):
        return i + (self.nx + 1) * (j + (self.ny + 1) * k)


def _node_grid(nx, ny, nz):
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1),
                          np.arange(nx + 1), indexing="ij")
    return i.ravel(), j.ravel(), k.ravel()


def mg_levels(nx: int, ny: int, nz: int, min_coarse: int = 2) -> int:
    """Largest level count l with every dim divisible by 2**(l-1) and the
    smallest coarse dim >= min_coarse (used when a workload omits l)."""
    l = 1
    while True:
        s = 2 ** l
        if nx % s or ny % s or nz % s or min(nx, ny, nz) // s < min_coarse:
            return l
        l += 1


def _mask_nodes(n_nodes, nodes):
    fixed = np.zeros(3 * n_nodes, dtype=np.uint8)
    nodes = np.asarray(nodes, dtype=np.int64)
    for c in range(3):
        fixed[3 * nodes + c] = 1
    return fixed


def _clamped_x0(nx, ny, nz):
    i, j, k = _node_grid(nx, ny, nz)
    nodes = np.nonzero(i == 0)[0]
    return _mask_nodes(i.size, nodes)


def _bottom_corners(nx, ny, nz):
    nn = (nx + 1) * (ny + 1) * (nz + 1)
    corners = [i + (nx + 1) * j for i in (0, nx) for j in (0, ny)]
    return _mask_nodes(nn, corners)


def cantilever_edge(nx, ny, nz, levels, V=None, vol_frac=0.3, load=-1.0,
                    rho_lo=1e-3, rho_hi=1.0, name=None) -> Problem:
    """Cantilever: face x=0 clamped; f_z = `load` at every node of the edge
    (x = nx, z = 0)."""
    fixed = _clamped_x0(nx, ny, nz)
    f = np.zeros(fixed.size)
    i, j, k = _node_grid(nx, ny, nz)
    edge = np.nonzero((i == nx) & (k == 0))[0]
    f[3 * edge + 2] = load
    f[fixed == 1] = 0.0
    m = nx * ny * nz
    V = vol_frac * m if V is None else V
    return Problem(name or f"cant-edge-{nx}x{ny}x{nz}-l{levels}", nx, ny, nz,
                   levels, fixed, f, float(V), rho_lo, rho_hi)


def cantilever_points(nx, ny, nz, levels, npoints=3, seed=0, V=None,
                      vol_frac=0.1, rho_lo=1e-3, rho_hi=1.0, name=None) -> Problem:
    """Cantilever with `npoints` unit -z nodal loads at distinct nodes (j, k)
    of the face x = nx, drawn uniformly with numpy's default_rng(seed);
    a colliding draw is redrawn."""
    fixed = _clamped_x0(nx, ny, nz)
    f = np.zeros(fixed.size)
    rng = np.random.default_rng(seed)
    picked: List[tuple] = []
    while len(picked) < npoints:
        jk = (int(rng.integers(0, ny + 1)), int(rng.integers(0, nz + 1)))
        if jk not in picked:
            picked.append(jk)
    for (j, k) in picked:
        p = nx + (nx + 1) * (j + (ny + 1) * k)
        f[3 * p + 2] = -1.0
    m = nx * ny * nz
    V = vol_frac * m if V is None else V
    pr = Problem(name or f"cant-points-{nx}x{ny}x{nz}-l{levels}", nx, ny, nz,
                 levels, fixed, f, float(V), rho_lo, rho_hi)
    pr.extra["load_nodes_jk"] = picked
    return pr


def point_cases(pr: Problem) -> np.ndarray:
    """The point loads of a `cantilever_points` problem as separate load
    cases, (npoints, n_dof)."""
    nx, ny = pr.nx, pr.ny
    cases = np.zeros((len(pr.extra["load_nodes_jk"]), pr.n_dof))
    for c, (j, k) in enumerate(pr.extra["load_nodes_jk"]):
        cases[c, 3 * (nx + (nx + 1) * (j + (ny + 1) * k)) + 2] = -1.0
    return cases


def load_cases(pr: Problem) -> np.ndarray:
    """The load cases of a problem as a (k, n_dof) array: the cases a
    multi-load problem carries, else its one load f."""
    cases = pr.extra.get("load_cases")
    if cases is None:
        return pr.f[None, :].copy()
    return np.asarray(cases, dtype=np.float64)


def with_load_cases(pr: Problem, cases, name=None) -> Problem:
    """A copy of `pr` with the given load cases (zeroed at fixed DOFs); its
    single load f is their sum."""
    cases = np.array(cases, dtype=np.float64).reshape(-1, pr.n_dof)
    cases[:, pr.fixed == 1] = 0.0
    out = Problem(name or pr.name + f"-k{cases.shape[0]}", pr.nx, pr.ny, pr.nz,
                  pr.levels, pr.fixed.copy(), cases.sum(axis=0), pr.V, pr.rho_lo,
                  pr.rho_hi, pr.E, pr.nu, pr.h, dict(pr.extra))
    out.extra["load_cases"] = cases
    return out


def cantilever_two_loads(nx, ny, nz, levels, vol_frac=0.3, rho_lo=1e-3,
                         rho_hi=1.0, name=None) -> Problem:
    """Cantilever (face x=0 clamped) with two load cases on its free end:
    f_z = -1 at every node of the edge (x = nx, z = 0), and f_y = -1 at
    every node of the edge (x = nx, z = nz)."""
    pr = cantilever_edge(nx, ny, nz, levels, vol_frac=vol_frac, rho_lo=rho_lo,
                         rho_hi=rho_hi)
    i, j, k = _node_grid(nx, ny, nz)
    second = np.zeros(pr.n_dof)
    edge = np.nonzero((i == nx) & (k == nz))[0]
    second[3 * edge + 1] = -1.0
    return with_load_cases(pr, [pr.f, second],
                           name or f"cant2load-{nx}x{ny}x{nz}-l{levels}")


def multi_config(idx: int) -> Problem:
    """Multi-load workloads (a sum of compliances over load cases):
    0: cantilever 16x8x8, 3 levels, the two end-edge load cases, V = 0.3 m
    1: cantilever 64x32x32, 5 levels, the two end-edge load cases, V = 0.2 m
    2: cantilever 192x96x96, 6 levels, the three seeded point loads of the
       benchmark's three-point cantilever as separate load cases, V = 0.1 m
    """
    if idx == 0:
        return cantilever_two_loads(16, 8, 8, 3, vol_frac=0.3, name="cant2load-16x8x8")
    if idx == 1:
        return cantilever_two_loads(64, 32, 32, 5, vol_frac=0.2, name="cant2load-64x32x32")
    if idx == 2:
        pr = cantilever_points(192, 96, 96, 6, npoints=3, seed=0, vol_frac=0.1)
        return with_load_cases(pr, point_cases(pr), name="cant3case-192x96x96")
    raise ValueError(idx)


def bridge_top(nx, ny, nz, levels, V=None, vol_frac=0.15, rho_lo=1e-3,
               rho_hi=1.0, name=None, h=1.0) -> Problem:
    """Bridge: the four bottom corners fixed; unit downward pressure on the
    whole top face z = nz, lumped to nodes as the consistent bilinear face
    load (each face of side h gives -h^2/4 to each of its 4 nodes).  With
    h = 2^(1 - levels) the domain is the coarse box of unit cubes refined
    levels - 1 times (the paper's BRIDGE-mx-my-mz-l domain), and the total
    load is the coarse top-face area at every refinement."""
    fixed = _bottom_corners(nx, ny, nz)
    f = np.zeros(fixed.size)
    i, j, k = _node_grid(nx, ny, nz)
    top = k == nz
    wx = np.where((i == 0) | (i == nx), 0.5, 1.0)
    wy = np.where((j == 0) | (j == ny), 0.5, 1.0)
    nodes = np.nonzero(top)[0]
    f[3 * nodes + 2] = -(h * h) * (wx * wy)[nodes]
    f[fixed == 1] = 0.0
    m = nx * ny * nz
    V = vol_frac * m if V is None else V
    return Problem(name or f"bridge-{nx}x{ny}x{nz}-l{levels}", nx, ny, nz,
                   levels, fixed, f, float(V), rho_lo, rho_hi, h=float(h))


def bar_rollers(nx, ny, nz, levels, vol_frac=0.5, traction=1.0,
                rho_lo=1e-3, rho_hi=1.0) -> Problem:
    """Prismatic bar on symmetry rollers (u_x = 0 on x = 0, u_y = 0 on y = 0,
    u_z = 0 on z = 0) pulled by a uniform axial traction on x = nx, lumped
    as the consistent bilinear face load.  Its displacement is a uniform
    strain for any uniform density, so every element carries the same
    energy (a test case with a known optimum)."""
    i, j, k = _node_grid(nx, ny, nz)
    fixed = np.zeros(3 * i.size, dtype=np.uint8)
    fixed[3 * np.nonzero(i == 0)[0] + 0] = 1
    fixed[3 * np.nonzero(j == 0)[0] + 1] = 1
    fixed[3 * np.nonzero(k == 0)[0] + 2] = 1
    f = np.zeros(fixed.size)
    wy = np.where((j == 0) | (j == ny), 0.5, 1.0)
    wz = np.where((k == 0) | (k == nz), 0.5, 1.0)
    face = np.nonzero(i == nx)[0]
    f[3 * face] = traction * (wy * wz)[face]
    f[fixed == 1] = 0.0
    m = nx * ny * nz
    return Problem(f"bar-{nx}x{ny}x{nz}-l{levels}", nx, ny, nz, levels, fixed,
                   f, vol_frac * m, rho_lo, rho_hi)


def paper_cantilever(mx, my, mz, l) -> Problem:
    """CANT-mx-my-mz-l of Section 7 (naming convention).  Only the mesh and
    the supports are defined by the paper; the load here is a unit -z force
    at the node nearest the middle of the face x = nx."""
    s = 2 ** (l - 1)
    nx, ny, nz = mx * s, my * s, mz * s
    fixed = _clamped_x0(nx, ny, nz)
    f = np.zeros(fixed.size)
    p = nx + (nx + 1) * (ny // 2 + (ny + 1) * (nz // 2))
    f[3 * p + 2] = -1.0
    return Problem(f"CANT-{mx}-{my}-{mz}-{l}", nx, ny, nz, l, fixed, f,
                   0.2 * nx * ny * nz, 0.0, 1.0)


def paper_bridge(mx, my, mz, l) -> Problem:
    """BRIDGE-mx-my-mz-l of Section 7 (mesh and supports as in the paper;
    load as in `bridge_top`)."""
    s = 2 ** (l - 1)
    pr = bridge_top(mx * s, my * s, mz * s, l, rho_lo=0.0, h=1.0 / s)
    pr.name = f"BRIDGE-{mx}-{my}-{mz}-{l}"
    return pr


def config(idx: int) -> Problem:
    """The benchmark workloads:
    0: cantilever 8x4x4, 3 levels, V = 0.3 m, FP64
    1: cantilever 64x32x32, 5 levels, V = 0.2 m, FP64, MINRES tol 1e-2
    2: bridge 128x64x64, 6 levels, V = 0.15 m, mixed precision, p floor 3e-3 |alpha|
    3: cantilever 192x96x96, 6 levels, 3 seeded point loads, V = 0.1 m, mixed
    """
    if idx == 0:
        pr = cantilever_edge(8, 4, 4, 3, vol_frac=0.3, name="cant-8x4x4")
        pr.extra.update(precision="fp64", eps_mr0=None)
    elif idx == 1:
        pr = cantilever_edge(64, 32, 32, 5, vol_frac=0.2, name="cant-64x32x32")
        pr.extra.update(precision="fp64", eps_mr0=1e-2)
    elif idx == 2:
        pr = bridge_top(128, 64, 64, 6, vol_frac=0.15, name="bridge-128x64x64",
                        h=2.0 ** -5)
        # the point-supported bridge needs a larger relative penalty floor for
        # the Gauss-Seidel multigrid to resolve its Newton systems
        pr.extra.update(precision="mixed", eps_mr0=None, p_min=3e-3)
    elif idx == 3:
        pr = cantilever_points(192, 96, 96, 6, npoints=3, seed=0,
                               vol_frac=0.1, name="cant3pt-192x96x96")
        pr.extra.update(precision="mixed", eps_mr0=None)
    else:
        raise ValueError(idx)
    return pr


CONFIGS = {0: "cant-8x4x4", 1: "cant-64x32x32", 2: "bridge-128x64x64",
           3: "cant3pt-192x96x96"}


def random_rho(m: int, seed: int = 1, lo: float = 1e-3, hi: float = 1.0):
    """Element densities ~ U[lo, hi], float64."""
    return np.random.default_rng(seed).uniform(lo, hi, size=m)


def random_vector(n: int, seed: int = 1, fixed: Optional[np.ndarray] = None):
    """Vector ~ U[-1, 1], float64, zeroed at fixed DOFs if a mask is given."""
    x = np.random.default_rng(seed).uniform(-1.0, 1.0, size=n)
    if fixed is not None:
        x[fixed[: n] == 1] = 0.0
    return x


SERVING_GRIDS = [(16, 8, 8, 3), (32, 16, 16, 4), (64, 32, 32, 5), (96, 48, 48, 5)]


def serving_requests(n_req: int = 256, rate: float = 1.0, seed: int = 0):
    """Poisson stream of VTS requests: grid uniform over SERVING_GRIDS, load
    kind uniform over {cantilever edge, bridge face}, V/m ~ U[0.1, 0.4].
    Returns a list of (arrival_time_s, Problem)."""
    root = np.random.default_rng(seed)
    ra, rs, rk, rv = (np.random.default_rng(s) for s in root.integers(0, 2**31, 4))
    t = np.cumsum(ra.exponential(1.0 / rate, size=n_req))
    out = []
    for r in range(n_req):
        nx, ny, nz, l = SERVING_GRIDS[int(rs.integers(0, len(SERVING_GRIDS)))]
        frac = float(rv.uniform(0.1, 0.4))
        if int(rk.integers(0, 2)) == 0:
            pr = cantilever_edge(nx, ny, nz, l, vol_frac=frac)
        else:
            pr = bridge_top(nx, ny, nz, l, vol_frac=frac, h=2.0 ** (1 - l))
        out.append((float(t[r]), pr))
    return out
