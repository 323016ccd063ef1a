"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This module only produces *inputs*: structured simplicial meshes (node
coordinates and P1 cell connectivity), Dirichlet masks and seeded nodal fields
(sources f, coefficients kappa).  It contains none of the finite element
arithmetic of the method (no element integrals, no tensors, no solves), so the
CPU oracle and the GPU path can both consume it without sharing method code.

Mesh conventions (fixed here because they change the tensor, not the matrix):
  * 1D  [0,1]:  node i at i/n, cells (i, i+1).
  * 2D  [0,1]^2: node (i,j) at (i/n, j/n) with id j*(n+1)+i; each square is
    split into the triangles (v00, v10, v11) and (v00, v11, v01).
  * 3D  [0,1]^3: node (i,j,k) with id (k*(n+1)+j)*(n+1)+i; each cube is split
    into 6 Kuhn (Freudenthal) tetrahedra: for every permutation p of the axes,
    v0 = corner, v_m = v_{m-1} + e_{p(m)}.
  * Dirichlet set: nodes with any coordinate equal to 0 or 1 (all of the
    boundary; the problems of the paper's results section use Gamma_D = Gamma).

Random numbers come from numpy's PCG64 (`numpy.random.default_rng(seed)`).
Workload seeds are 20050619 + workload index (1..5); instance m of the batched
workload adds 1000*m.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_BASE = 20050619


# ----------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------
@dataclass
class Mesh:
    dim: int
    n: int                      # subdivisions per axis
    coords: np.ndarray          # float64 [N, dim]
    cells: np.ndarray           # int32   [E, dim+1]
    dirichlet: np.ndarray       # uint8   [N], 1 on the boundary

    @property
    def n_nodes(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_cells(self) -> int:
        return int(self.cells.shape[0])


def mesh_1d(n: int) -> Mesh:
    i = np.arange(n + 1)
    coords = (i / n).astype(np.float64)[:, None]
    cells = np.stack([np.arange(n), np.arange(1, n + 1)], axis=1).astype(np.int32)
    mask = ((i == 0) | (i == n)).astype(np.uint8)
    return Mesh(1, n, coords, cells, mask)


def mesh_2d(n: int) -> Mesh:
    m = n + 1
    jj, ii = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    ii = ii.ravel()
    jj = jj.ravel()
    coords = np.stack([ii / n, jj / n], axis=1).astype(np.float64)
    ci, cj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ci = ci.ravel()
    cj = cj.ravel()
    v00 = cj * m + ci
    v10 = v00 + 1
    v01 = v00 + m
    v11 = v01 + 1
    t1 = np.stack([v00, v10, v11], axis=1)
    t2 = np.stack([v00, v11, v01], axis=1)
    cells = np.empty((2 * n * n, 3), dtype=np.int32)
    cells[0::2] = t1
    cells[1::2] = t2
    mask = ((ii == 0) | (ii == n) | (jj == 0) | (jj == n)).astype(np.uint8)
    return Mesh(2, n, coords, cells, mask)


def mesh_3d(n: int) -> Mesh:
    m = n + 1
    kk, jj, ii = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    ii = ii.ravel()
    jj = jj.ravel()
    kk = kk.ravel()
    coords = np.stack([ii / n, jj / n, kk / n], axis=1).astype(np.float64)
    ck, cj, ci = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    corner = (ck.ravel() * m + cj.ravel()) * m + ci.ravel()
    stride = np.array([1, m, m * m])
    tets = []
    for perm in itertools.permutations(range(3)):
        v0 = corner
        v1 = v0 + stride[perm[0]]
        v2 = v1 + stride[perm[1]]
        v3 = v2 + stride[perm[2]]
        tets.append(np.stack([v0, v1, v2, v3], axis=1))
    cells = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    mask = ((ii == 0) | (ii == n) | (jj == 0) | (jj == n) | (kk == 0) | (kk == n)).astype(np.uint8)
    return Mesh(3, n, coords, cells, mask)


def structured_mesh(dim: int, n: int) -> Mesh:
    return {1: mesh_1d, 2: mesh_2d, 3: mesh_3d}[dim](n)


# ----------------------------------------------------------------------------
# seeded nodal fields
# ----------------------------------------------------------------------------
def gaussian_sum(coords: np.ndarray, rng: np.random.Generator, count: int = 8,
                 amp=(1.0, 20.0), width=(0.05, 0.2)) -> np.ndarray:
    """Sum of `count` isotropic Gaussians A exp(-|x-c|^2 / (2 s^2)) at the nodes;
    A ~ U[amp], s ~ U[width], centres c ~ U[0,1]^dim."""
    dim = coords.shape[1]
    A = rng.uniform(amp[0], amp[1], size=count)
    s = rng.uniform(width[0], width[1], size=count)
    c = rng.uniform(0.0, 1.0, size=(count, dim))
    out = np.zeros(coords.shape[0], dtype=np.float64)
    for m in range(count):
        d2 = np.sum((coords - c[m]) ** 2, axis=1)
        out += A[m] * np.exp(-d2 / (2.0 * s[m] ** 2))
    return out


def grid_smooth(values: np.ndarray, dim: int, n: int, sweeps: int) -> np.ndarray:
    """Damped Jacobi sweeps (weight 2/3) on the grid graph Laplacian with natural
    (Neumann) ends: v <- v - (2/3) (deg v - sum_nbr v) / deg.  A generic
    smoothing of seeded noise on the structured node grid."""
    shape = (n + 1,) * dim
    v = values.reshape(shape[::-1]).copy()   # axes ordered (.., j, i)
    for _ in range(sweeps):
        nbr_sum = np.zeros_like(v)
        deg = np.zeros_like(v)
        for ax in range(dim):
            sl_lo = [slice(None)] * dim
            sl_hi = [slice(None)] * dim
            sl_lo[ax] = slice(0, -1)
            sl_hi[ax] = slice(1, None)
            nbr_sum[tuple(sl_lo)] += v[tuple(sl_hi)]
            nbr_sum[tuple(sl_hi)] += v[tuple(sl_lo)]
            deg[tuple(sl_lo)] += 1.0
            deg[tuple(sl_hi)] += 1.0
        v = v - (2.0 / 3.0) * (deg * v - nbr_sum) / deg
    return v.reshape(-1)


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------
FORM_STIFF = 0   # T_ijk = int psi_k grad phi_j . grad phi_i
FORM_MASS = 1    # T_ijk = int phi_k phi_j phi_i
FORM_CONV = 2    # T_ijk = int phi_k phi_j (sum_d d/dx_d phi_i)


@dataclass
class Workload:
    name: str
    mesh: Mesh
    f: np.ndarray                   # nodal source values [N]; load b = M f
    form: int                       # FORM_STIFF or FORM_MASS
    a0: Optional[np.ndarray]        # nodal a0 field [N] or None (then a0_const)
    a0_const: float                 # a = a0 + u^2
    add_stiffness: bool             # residual gets + K u (semilinear form)
    tol: float                      # Newton tolerance on ||F|| / ||F_0||
    seed: int
    extra: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return self.mesh.n_nodes


def nonlinear_diffusion_1d(n: int = 256, seed: int = SEED_BASE + 1) -> Workload:
    """-((1+u^2) u')' = f on [0,1], u(0)=u(1)=0, f nodal ~ U[0,10]."""
    rng = np.random.default_rng(seed)
    mesh = mesh_1d(n)
    f = rng.uniform(0.0, 10.0, size=mesh.n_nodes)
    return Workload(f"nonlinear_diffusion_1d_n{n}", mesh, f, FORM_STIFF, None, 1.0,
                    False, 1e-12, seed)


def nonlinear_diffusion_2d(n: int = 256, seed: int = SEED_BASE + 2) -> Workload:
    """-div((1+u^2) grad u) = f on the unit square, zero Dirichlet data,
    f = sum of 8 seeded Gaussians."""
    rng = np.random.default_rng(seed)
    mesh = mesh_2d(n)
    f = gaussian_sum(mesh.coords, rng)
    return Workload(f"nonlinear_diffusion_2d_n{n}", mesh, f, FORM_STIFF, None, 1.0,
                    False, 1e-10, seed)


def semilinear_2d(n: int = 512, seed: int = SEED_BASE + 3) -> Workload:
    """-Laplace(u) + u^3 = f on the unit square, zero Dirichlet data,
    f = U[-50,50] nodal noise smoothed by 2 damped Jacobi sweeps.
    u^3 = u * w with w = u^2 on P1 (mass tensor), plus the stiffness matrix."""
    rng = np.random.default_rng(seed)
    mesh = mesh_2d(n)
    noise = rng.uniform(-50.0, 50.0, size=mesh.n_nodes)
    f = grid_smooth(noise, 2, n, 2)
    return Workload(f"semilinear_2d_n{n}", mesh, f, FORM_MASS, None, 0.0,
                    True, 1e-10, seed)


def batch_sizes(count: int = 64, seed: int = SEED_BASE + 4, lo: int = 32, hi: int = 256) -> List[int]:
    rng = np.random.default_rng(seed)
    return [int(x) for x in rng.integers(lo, hi + 1, size=count)]


def nonlinear_diffusion_batch(count: int = 64, seed: int = SEED_BASE + 4,
                              lo: int = 32, hi: int = 256) -> List[Workload]:
    """`count` independent 2D nonlinear-diffusion instances, n ~ U{lo..hi},
    each with its own Gaussian-sum source (seed + 1000*m)."""
    out = []
    for m, n in enumerate(batch_sizes(count, seed, lo, hi)):
        w = nonlinear_diffusion_2d(n, seed + 1000 * (m + 1))
        w.name = f"batch{m}_n{n}"
        out.append(w)
    return out


def smooth_log_field(mesh: Mesh, rng: np.random.Generator, lo: float, hi: float,
                     sweeps: int = 4) -> np.ndarray:
    """exp of smoothed seeded noise, min-max mapped into [ln lo, ln hi]."""
    noise = rng.uniform(-1.0, 1.0, size=mesh.n_nodes)
    s = grid_smooth(noise, mesh.dim, mesh.n, sweeps)
    s = (s - s.min()) / (s.max() - s.min())
    return np.exp(np.log(lo) + s * (np.log(hi) - np.log(lo)))


def diffusion_3d(n: int = 64, seed: int = SEED_BASE + 5) -> Workload:
    """-div((kappa+u^2) grad u) = f on the unit cube (Kuhn tetrahedra), zero
    Dirichlet data; kappa = exp(smooth noise) in [0.5, 2]; f = 8 Gaussians.
    extra['f_target'] is a second seeded source whose solution is the tracking
    target u_d of the objective 0.5 ||u - u_d||^2."""
    rng = np.random.default_rng(seed)
    mesh = mesh_3d(n)
    kappa = smooth_log_field(mesh, rng, 0.5, 2.0)
    f = gaussian_sum(mesh.coords, rng)
    f_target = gaussian_sum(mesh.coords, rng)
    return Workload(f"diffusion_3d_n{n}", mesh, f, FORM_STIFF, kappa, 0.0, False, 1e-13,
                    seed, extra={"f_target": f_target})


def direction(n_nodes: int, seed: int) -> np.ndarray:
    """Seeded U[-1,1] direction for finite-difference checks."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n_nodes)


# ----------------------------------------------------------------------------
# viscous Burgers' equation with a manufactured solution (the time-dependent
# benchmark of the paper's results section)
# ----------------------------------------------------------------------------
def burgers_exact(x1: np.ndarray, x2: np.ndarray, t: float) -> np.ndarray:
    """u(x, t) = 10 x1 x2 (x1-1)(x2-1) [sin(2 x1 t) e^{-t/2} + cos(x2 t) e^{-t/4}
    + sin(x1 x2 t) e^{-t}] on the unit square; zero on its boundary."""
    P = 10.0 * x1 * x2 * (x1 - 1.0) * (x2 - 1.0)
    S = (np.sin(2.0 * x1 * t) * np.exp(-0.5 * t) + np.cos(x2 * t) * np.exp(-0.25 * t)
         + np.sin(x1 * x2 * t) * np.exp(-t))
    return P * S


def burgers_source(x1: np.ndarray, x2: np.ndarray, t: float, nu: float) -> np.ndarray:
    """d = u_t - nu (u_11 + u_22) + u (u_1 + u_2) for u = burgers_exact, by the
    product rule on u = P S (P the polynomial factor, S the bracket)."""
    e1, e2, e3 = math.exp(-0.5 * t), math.exp(-0.25 * t), math.exp(-t)
    s1, c1 = np.sin(2.0 * x1 * t), np.cos(2.0 * x1 * t)
    s2, c2 = np.sin(x2 * t), np.cos(x2 * t)
    s3, c3 = np.sin(x1 * x2 * t), np.cos(x1 * x2 * t)
    S = s1 * e1 + c2 * e2 + s3 * e3
    S_t = (2.0 * x1 * c1 - 0.5 * s1) * e1 + (-x2 * s2 - 0.25 * c2) * e2 + (x1 * x2 * c3 - s3) * e3
    S_1 = 2.0 * t * c1 * e1 + x2 * t * c3 * e3
    S_2 = -t * s2 * e2 + x1 * t * c3 * e3
    S_11 = -4.0 * t * t * s1 * e1 - x2 * x2 * t * t * s3 * e3
    S_22 = -t * t * c2 * e2 - x1 * x1 * t * t * s3 * e3
    P = 10.0 * x1 * x2 * (x1 - 1.0) * (x2 - 1.0)
    P_1 = 10.0 * x2 * (x2 - 1.0) * (2.0 * x1 - 1.0)
    P_2 = 10.0 * x1 * (x1 - 1.0) * (2.0 * x2 - 1.0)
    P_11 = 20.0 * x2 * (x2 - 1.0)
    P_22 = 20.0 * x1 * (x1 - 1.0)
    u = P * S
    u_t = P * S_t
    u_1 = P_1 * S + P * S_1
    u_2 = P_2 * S + P * S_2
    lap = P_11 * S + 2.0 * P_1 * S_1 + P * S_11 + P_22 * S + 2.0 * P_2 * S_2 + P * S_22
    return u_t - nu * lap + u * (u_1 + u_2)


@dataclass
class BurgersWorkload:
    name: str
    mesh: Mesh
    dt: float
    nu: float
    steps: int
    u0: np.ndarray                  # nodal initial value [N]
    source: np.ndarray              # nodal source values at t_1..t_steps [steps, N]
    u_final: np.ndarray             # exact solution at t_steps, nodal [N]

    @property
    def n_nodes(self) -> int:
        return self.mesh.n_nodes


def burgers_2d(n: int = 256, dt: float = 1e-2, t_end: float = 1.0, nu: float = 1.0) -> BurgersWorkload:
    """Viscous 2D Burgers' equation u_t - nu Lap u + u u_1 + u u_2 = d on the
    unit square, zero Dirichlet data, source and initial value of the
    manufactured solution burgers_exact; nu = 1, T = 1, dt = 1e-2 as in the
    paper's experiment.  Deterministic (no random numbers)."""
    mesh = mesh_2d(n)
    steps = int(round(t_end / dt))
    x1, x2 = mesh.coords[:, 0], mesh.coords[:, 1]
    u0 = burgers_exact(x1, x2, 0.0)
    src = np.stack([burgers_source(x1, x2, (m + 1) * dt, nu) for m in range(steps)])
    return BurgersWorkload(f"burgers_2d_n{n}_dt{dt:g}", mesh, dt, nu, steps, u0, src,
                           burgers_exact(x1, x2, steps * dt))


# ----------------------------------------------------------------------------
# p-Laplace equation on the unit disk (the gradient-nonlinearity benchmark of
# the paper's results section)
# ----------------------------------------------------------------------------
def mesh_disk(n: int) -> Mesh:
    """Unit disk: the 2D mesh of [-1,1]^2 with n x n squares (same numbering and
    diagonals as mesh_2d) mapped by (x, y) -> (x sqrt(1 - y^2/2), y sqrt(1 - x^2/2)),
    which takes the square's boundary onto the circle; Dirichlet = boundary."""
    m = mesh_2d(n)
    x = 2.0 * m.coords[:, 0] - 1.0
    y = 2.0 * m.coords[:, 1] - 1.0
    c = np.stack([x * np.sqrt(1.0 - 0.5 * y * y), y * np.sqrt(1.0 - 0.5 * x * x)], axis=1)
    return Mesh(2, n, c, m.cells, m.dirichlet)


def plaplace_exact(coords: np.ndarray, p: float) -> np.ndarray:
    """Radial solution of -div(|grad u|^{p-2} grad u) = 1 on the unit disk, u = 0
    on the circle: u = 2^{-1/(p-1)} (p-1)/p (1 - |x|^{p/(p-1)})."""
    r = np.sqrt(np.sum(coords * coords, axis=1))
    return 2.0 ** (-1.0 / (p - 1.0)) * (p - 1.0) / p * (1.0 - r ** (p / (p - 1.0)))


@dataclass
class GradientWorkload:
    name: str
    mesh: Mesh
    f: np.ndarray                   # nodal source values; load M f
    p: float                        # coefficient (c0 + c1 |grad u|^2)^q with
    c0: float                       #   p-Laplace: c0 = eps^2, c1 = 1, q = (p - 2) / 2
    c1: float
    q: float
    exact: Optional[np.ndarray]     # nodal exact solution or None

    @property
    def n_nodes(self) -> int:
        return self.mesh.n_nodes


def plaplace_disk(n: int = 256, p: float = 1.5, eps: float = 0.0) -> GradientWorkload:
    """p-Laplace on the unit disk with source 1 (p = 3/2 as in the paper)."""
    m = mesh_disk(n)
    return GradientWorkload(f"plaplace_disk_n{n}_p{p:g}", m, np.ones(m.n_nodes), p, eps * eps, 1.0,
                            (p - 2.0) / 2.0, plaplace_exact(m.coords, p))


WORKLOADS = {
    "1d": nonlinear_diffusion_1d,
    "2d": nonlinear_diffusion_2d,
    "2d_semilinear": semilinear_2d,
    "3d": diffusion_3d,
}
