"""Plain FP64 CPU oracle for the EGFEM Newton hot path -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module.  The product path (the HIP library and its Python
binding) never calls it, and it shares no code with that path: the only thing
both sides consume is the seeded input module `workloads`.

What is computed, in the paper's notation (Tolle & Marheineke, "Extended Group
Finite Element Method", arXiv 2005.06193):

* Sec. 2.1 / eq. (discrete_problem): P1 Lagrange trial space V_h on a simplicial
  mesh, Dirichlet nodes fixed (here u_D = 0), one equation per free node.
* Sec. 3.3 / eq. (egfem_terms): with b(u) = u the trilinear form
  K_a : (u (x) a) uses the third-order tensor
      (K_a)_ijk = int eta_k grad phi_j . grad phi_i          (stiffness form)
  and, for the semilinear example of Sec. 5.3 decomposition (a),
      (M_c)_ijk = int eta_k phi_j phi_i                      (mass form).
  The nonlinearity is interpolated onto W_h = V_h = P1 (Case 2 of Sec. 3.1,
  the original group FEM choice), so eta_k = phi_k and the interpolation
  operator Pi_u of Sec. 3.2 is the identity.
* Sec. 4 / eq. (EGFEM_root) reduced to u: F(u) = [K u] + T:(u (x) a(u)) - d
  with a(u) = a0 + u*u evaluated pointwise at the nodes (eq. egfem_coeffs).
* Sec. 4, Picard iteration (Example picard_iteration): u^{n+1} solves
  ([K] + T . a(u^n)) u^{n+1} = d, then a is updated pointwise.
* Sec. 4, Newton iteration: u <- u - DF(u)^{-1} F(u).  The Jacobian needs no
  integration: DF = [K] + T . a + (T ._2 u) diag(a'(u)), the contractions of
  the Notation in Sec. 3.3.  The lifted iteration on z = (u, a) with the block
  Jacobian printed in Sec. 4 is implemented as well (dense, tiny meshes).
* Sec. 2.1 eq. (nonlinear_terms) and eq. (SGA_root): the standard Galerkin
  approach, re-integrating the nonlinear term by quadrature every iteration.
* Sec. 3.1 Case 1 / Example exact_egfem: W_h = P2 makes the reformulation
  exact (EGFEM(P2) == SGA for the u^2 nonlinearity).
* Sec. 3.1 Case 3: W_h = I_k, the coefficient carried at the points of a
  quadrature rule (Pi_u evaluates the P1 iterate there); with a rule exact for
  the integrand this is again the standard Galerkin approach.
* Sec. 3.2 gradient interpolation with W_h = P0 (the p-Laplace and minimal
  surface examples of Sec. 5): a(grad u) per cell, T_ijk = K^{e_k}_ij, Picard.
* Sec. 5.2, Burgers' equation: the convection tensor
  N_ijk = int phi_k phi_j (d_1 + d_2) phi_i and the semi-implicit time step
  (M + dt nu K) u^{n+1} = M u^n + dt (1/2 N:(u^n (x) u^n) + d^{n+1}), in the
  tensor and the group (N^f (u . u)) formulations, the latter also with
  W_h = P2 and W_h = I_k (f = (Pi_u u)^2 at the P2 dofs or the points).

Integrals use numerical quadrature on the reference simplex (collapsed Gauss-
Legendre product rules generated here), assembled element by element.  Linear
systems are solved directly (SuperLU through scipy) -- the plain definition of
"solve J delta = -F".  Everything is float64.

Readings of points the paper leaves open are listed in the project's design
notes; the ones that change numbers are: load d = M f for a nodal source f;
Newton stops on ||F||_2 <= tol ||F(u0)||_2 over the free rows; damping halves
the step up to 10 times while ||F(u + alpha delta)|| > (1 - 1e-4 alpha) ||F(u)||;
assembled tensor entries below 1e-13 of their row's largest magnitude (zero
in exact arithmetic) are dropped.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

FORM_STIFF = 0
FORM_MASS = 1
FORM_CONV = 2


# ----------------------------------------------------------------------------
# quadrature on the reference simplex {x_m >= 0, sum x_m <= 1}
# ----------------------------------------------------------------------------
def gauss_legendre_01(m: int):
    """m-point Gauss-Legendre rule on [0,1] (exact for degree 2m-1)."""
    x, w = np.polynomial.legendre.leggauss(m)
    return 0.5 * (x + 1.0), 0.5 * w


def simplex_quadrature(dim: int, degree: int):
    """Collapsed (Duffy) Gauss-Legendre product rule on the reference simplex,
    exact for polynomials of total degree <= `degree`.  Returns points [Q, dim]
    and weights [Q] summing to the reference volume 1/dim!.

    Map from the unit cube: x1 = s1, x2 = s2 (1 - s1), x3 = s3 (1 - s1)(1 - s2),
    Jacobian (1-s1)^(dim-1) (1-s2)^(dim-2).  A degree-q polynomial becomes a
    polynomial of degree <= q + dim - 1 in each cube variable, so each axis
    takes ceil((q + dim) / 2) Gauss points.
    """
    m = max(1, math.ceil((degree + dim) / 2))
    s, w = gauss_legendre_01(m)
    if dim == 1:
        return s[:, None].copy(), w.copy()
    grids = np.meshgrid(*([s] * dim), indexing="ij")
    wgrids = np.meshgrid(*([w] * dim), indexing="ij")
    S = np.stack([g.ravel() for g in grids], axis=1)
    W = np.prod(np.stack([g.ravel() for g in wgrids], axis=1), axis=1)
    X = np.zeros_like(S)
    scale = np.ones(S.shape[0])
    for ax in range(dim):
        X[:, ax] = S[:, ax] * scale
        scale = scale * (1.0 - S[:, ax])
    jac = np.ones(S.shape[0])
    for ax in range(dim - 1):
        jac = jac * (1.0 - S[:, ax]) ** (dim - 1 - ax)
    return X, W * jac


def barycentric(points: np.ndarray) -> np.ndarray:
    """Barycentric coordinates [Q, dim+1] of reference points: lambda_0 = 1 - sum x,
    lambda_m = x_m.  These are the P1 nodal basis functions on the element."""
    return np.concatenate([1.0 - points.sum(axis=1, keepdims=True), points], axis=1)


# ----------------------------------------------------------------------------
# element geometry
# ----------------------------------------------------------------------------
def element_geometry(coords: np.ndarray, cells: np.ndarray):
    """B_e = [x1-x0, ..., xd-x0], |det B_e| and the (constant) gradients of the
    barycentric basis functions G[e, a, :] = grad lambda_a."""
    X = coords[cells]                       # [E, d+1, d]
    dim = X.shape[2]
    B = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))   # columns x_m - x_0
    if dim == 1:
        det = B[:, 0, 0].copy()
        Binv = 1.0 / B
    else:
        det = np.linalg.det(B)
        Binv = np.linalg.inv(B)
    if np.any(det == 0.0):
        raise ValueError("degenerate element")
    # lambda_m (m>=1) = row m-1 of B^{-1} applied to (x - x0)
    G = np.empty((X.shape[0], dim + 1, dim))
    G[:, 1:, :] = Binv
    G[:, 0, :] = -Binv.sum(axis=1)
    return np.abs(det), G


# ----------------------------------------------------------------------------
# sparse third-order tensor in coordinate form
# ----------------------------------------------------------------------------
@dataclass
class Tensor3:
    n: int
    i: np.ndarray
    j: np.ndarray
    k: np.ndarray
    v: np.ndarray
    structural_nnz: int = 0

    @property
    def nnz(self) -> int:
        return int(self.v.size)

    def dense(self) -> np.ndarray:
        D = np.zeros((self.n, self.n, self.n))
        np.add.at(D, (self.i, self.j, self.k), self.v)
        return D


DROP_REL = 1e-13


def _merge_coo3(n, I, J, K, V, drop_rel=DROP_REL) -> Tensor3:
    """Sum duplicate (i,j,k) entries in element order, then drop the entries that
    vanish in exact arithmetic: |T_ijk| <= drop_rel * max_{j',k'} |T_ij'k'| (row-
    relative; with drop_rel = 0 only exact 0.0 is dropped).  On right-isosceles
    triangles and Kuhn tetrahedra grad phi_i . grad phi_j = 0 for some vertex
    pairs; rounding turns these into a few ulps when h is not a power of two."""
    key = (I.astype(np.int64) * n + J) * n + K
    order = np.argsort(key, kind="stable")
    key = key[order]
    V = V[order]
    starts = np.flatnonzero(np.concatenate([[True], key[1:] != key[:-1]]))
    vals = np.add.reduceat(V, starts) if V.size else V
    ukey = key[starts]
    structural = int(ukey.size)
    i = ukey // (n * n)
    rowmax = np.zeros(n)
    np.maximum.at(rowmax, i, np.abs(vals))
    keep = np.abs(vals) > drop_rel * rowmax[i]
    keep &= vals != 0.0
    ukey = ukey[keep]
    vals = vals[keep]
    i = ukey // (n * n)
    j = (ukey // n) % n
    k = ukey % n
    return Tensor3(n, i, j, k, vals, structural)


def _degree_for(form: int, dim: int) -> int:
    # stiffness integrand eta_k grad.grad is linear; convection integrand
    # phi_k phi_j (grad phi_i . 1) quadratic; mass integrand cubic
    return {FORM_STIFF: 1, FORM_MASS: 3, FORM_CONV: 2}[form]


def assemble_tensor(coords, cells, form: int, degree: Optional[int] = None,
                    drop_rel: float = DROP_REL) -> Tensor3:
    """T_ijk = sum_e sum_q w_q |det B_e| psi_k(x_q) grad phi_j . grad phi_i   (stiffness)
    or T_ijk = sum_e sum_q w_q |det B_e| psi_k phi_j phi_i (x_q)              (mass)
    or T_ijk = sum_e sum_q w_q |det B_e| phi_k phi_j (x_q) sum_d d_d phi_i    (convection,
    the tensor N of the Burgers example, Sec. 5.2),
    with psi = phi = P1 nodal basis (eq. egfem_terms, Case 2 with W_h = V_h)."""
    n = coords.shape[0]
    dim = coords.shape[1]
    if degree is None:
        degree = _degree_for(form, dim)
    det, G = element_geometry(coords, cells)
    pts, wts = simplex_quadrature(dim, degree)
    lam = barycentric(pts)                                   # [Q, d+1]
    if form == FORM_STIFF:
        GG = np.einsum("ead,ebd->eab", G, G)                 # grad phi_a . grad phi_b
        psi = np.einsum("q,qc->c", wts, lam)                 # int over reference of psi_c
        Te = det[:, None, None, None] * GG[:, :, :, None] * psi[None, None, None, :]
    elif form == FORM_MASS:
        trip = np.einsum("q,qa,qb,qc->abc", wts, lam, lam, lam)
        Te = det[:, None, None, None] * trip[None]
    elif form == FORM_CONV:
        gsum = G.sum(axis=2)                                 # sum_d d_d phi_a, [E, d+1]
        # a sum that vanishes in exact arithmetic (middle vertices of Kuhn
        # tetrahedra) is zero, not rounding noise: the exact-zero drop rule
        gsum[np.abs(gsum) <= 1e-12 * np.abs(G).sum(axis=2)] = 0.0
        pair = np.einsum("q,qb,qc->bc", wts, lam, lam)       # int over reference of phi_b phi_c
        Te = det[:, None, None, None] * gsum[:, :, None, None] * pair[None, None]
    else:
        raise ValueError("unknown form")
    nl = dim + 1
    a_idx, b_idx, c_idx = np.meshgrid(np.arange(nl), np.arange(nl), np.arange(nl), indexing="ij")
    I = cells[:, a_idx.ravel()].ravel().astype(np.int64)
    J = cells[:, b_idx.ravel()].ravel().astype(np.int64)
    K = cells[:, c_idx.ravel()].ravel().astype(np.int64)
    return _merge_coo3(n, I, J, K, Te.reshape(-1), drop_rel)


def assemble_stiffness(coords, cells) -> sp.csr_matrix:
    """K_ij = int grad phi_j . grad phi_i."""
    n = coords.shape[0]
    det, G = element_geometry(coords, cells)
    dim = coords.shape[1]
    vol = det / math.factorial(dim)
    Ke = vol[:, None, None] * np.einsum("ead,ebd->eab", G, G)
    return _scatter_matrix(n, cells, Ke)


def assemble_mass(coords, cells) -> sp.csr_matrix:
    """M_ij = int phi_j phi_i, by quadrature of degree 2."""
    n = coords.shape[0]
    dim = coords.shape[1]
    det, _ = element_geometry(coords, cells)
    pts, wts = simplex_quadrature(dim, 2)
    lam = barycentric(pts)
    Me = det[:, None, None] * np.einsum("q,qa,qb->ab", wts, lam, lam)[None]
    return _scatter_matrix(n, cells, Me)


def _scatter_matrix(n, cells, Ae) -> sp.csr_matrix:
    nl = cells.shape[1]
    rows = np.repeat(cells, nl, axis=1).ravel()
    cols = np.tile(cells, (1, nl)).ravel()
    A = sp.coo_matrix((Ae.reshape(-1), (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    return A


# ----------------------------------------------------------------------------
# tensor contractions (Notation, Sec. 3.3)
# ----------------------------------------------------------------------------
def contract_uv(T: Tensor3, u: np.ndarray, a: np.ndarray) -> np.ndarray:
    """(T : (u (x) a))_i = sum_jk T_ijk u_j a_k."""
    return np.bincount(T.i, weights=T.v * u[T.j] * a[T.k], minlength=T.n)


def contract_first(T: Tensor3, a: np.ndarray) -> sp.csr_matrix:
    """(T . a)_ij = sum_k T_ijk a_k."""
    return sp.coo_matrix((T.v * a[T.k], (T.i, T.j)), shape=(T.n, T.n)).tocsr()


def contract_mode2(T: Tensor3, u: np.ndarray) -> sp.csr_matrix:
    """(T ._2 u)_ik = sum_j T_ijk u_j."""
    return sp.coo_matrix((T.v * u[T.j], (T.i, T.k)), shape=(T.n, T.n)).tocsr()


def contract_mode3(T: Tensor3, lam: np.ndarray, u: np.ndarray) -> np.ndarray:
    """x_k = sum_ij lam_i T_ijk u_j (adjoint of the a-dependence)."""
    return np.bincount(T.k, weights=T.v * lam[T.i] * u[T.j], minlength=T.n)


# ----------------------------------------------------------------------------
# problem definition and the reduced EGFEM Newton iteration
# ----------------------------------------------------------------------------
@dataclass
class Problem:
    T: Tensor3
    d: np.ndarray                  # load vector (the paper's d), d = M f
    dirichlet: np.ndarray          # bool [N]
    a0: np.ndarray                 # [N]
    K: Optional[sp.csr_matrix] = None   # added linear stiffness (semilinear form)
    M: Optional[sp.csr_matrix] = None
    coords: Optional[np.ndarray] = None
    cells: Optional[np.ndarray] = None
    form: int = FORM_STIFF

    @property
    def n(self) -> int:
        return self.T.n

    @property
    def free(self) -> np.ndarray:
        return ~self.dirichlet


def build_problem(workload, degree: Optional[int] = None, drop_rel: float = DROP_REL) -> Problem:
    """Offline phase: tensor, matrices and load for a workload from `workloads`."""
    mesh = workload.mesh
    T = assemble_tensor(mesh.coords, mesh.cells, workload.form, degree, drop_rel)
    M = assemble_mass(mesh.coords, mesh.cells)
    K = assemble_stiffness(mesh.coords, mesh.cells) if workload.add_stiffness else None
    a0 = (np.asarray(workload.a0, dtype=np.float64).copy() if workload.a0 is not None
          else np.full(mesh.n_nodes, float(workload.a0_const)))
    d = M @ workload.f
    return Problem(T, d, mesh.dirichlet.astype(bool), a0, K, M, mesh.coords, mesh.cells,
                   workload.form)


def nodal_a(p: Problem, u: np.ndarray) -> np.ndarray:
    """a = a0 + u*u at the W-dofs (eq. egfem_coeffs with Pi_u = identity)."""
    return p.a0 + u * u


def nodal_da(p: Problem, u: np.ndarray) -> np.ndarray:
    """pointwise derivative a'(u) = 2u."""
    return 2.0 * u


def residual(p: Problem, u: np.ndarray) -> np.ndarray:
    """F(u) = [K u] + T:(u (x) a(u)) - d, Dirichlet rows set to zero."""
    F = contract_uv(p.T, u, nodal_a(p, u)) - p.d
    if p.K is not None:
        F = F + p.K @ u
    F[p.dirichlet] = 0.0
    return F


def residual_elementwise(p: Problem, u: np.ndarray, rows: Optional[np.ndarray] = None) -> np.ndarray:
    """The same F(u) evaluated without the global tensor: per element,
    (T:(u (x) a))_i = int a_h grad u_h . grad phi_i  (stiffness form) or
    int a_h u_h phi_i (mass form) with a_h the P1 interpolant of a = a0 + u^2
    (the group-FEM product approximation of Sec. 2.2), by quadrature.
    With `rows`, only the cells touching those nodes are visited and only
    F[rows] is meaningful."""
    coords, cells = p.coords, p.cells
    if rows is not None:
        touch = np.zeros(p.n, dtype=bool)
        touch[rows] = True
        cells = cells[touch[cells].any(axis=1)]
    dim = coords.shape[1]
    det, G = element_geometry(coords, cells)
    a = nodal_a(p, u)
    ae = a[cells]
    ue = u[cells]
    if p.form == FORM_STIFF:
        pts, wts = simplex_quadrature(dim, 1)
        lam = barycentric(pts)
        c = det * ((ae @ lam.T) @ wts)                       # int a_h over the element
        gu = np.einsum("ea,ead->ed", ue, G)
        Re = c[:, None] * np.einsum("ead,ed->ea", G, gu)
    else:
        pts, wts = simplex_quadrature(dim, 3)
        lam = barycentric(pts)
        wq = det[:, None] * wts[None, :]
        Re = np.einsum("eq,qa->ea", wq * (ae @ lam.T) * (ue @ lam.T), lam)
    F = np.bincount(cells.ravel(), weights=Re.ravel(), minlength=p.n) - p.d
    if p.K is not None:
        F = F + p.K @ u
    F[p.dirichlet] = 0.0
    return F


def tensor_rows(p_or_mesh_coords, cells, form: int, rows: np.ndarray,
                drop_rel: float = DROP_REL) -> Tensor3:
    """The stored entries T_ijk for i in `rows` only, assembled from the cells
    that touch those nodes (every contribution to row i comes from a cell
    containing node i), for spot checks at full size."""
    coords = p_or_mesh_coords
    n = coords.shape[0]
    touch = np.zeros(n, dtype=bool)
    touch[rows] = True
    sub = cells[touch[cells].any(axis=1)]
    T = assemble_tensor(coords, sub, form, drop_rel=drop_rel)
    keep = touch[T.i]
    return Tensor3(n, T.i[keep], T.j[keep], T.k[keep], T.v[keep])


def _apply_dirichlet(p: Problem, J: sp.csr_matrix) -> sp.csr_matrix:
    free = sp.diags(p.free.astype(np.float64))
    dirm = sp.diags(p.dirichlet.astype(np.float64))
    return (free @ J @ free + dirm).tocsr()


def jacobian(p: Problem, u: np.ndarray) -> sp.csr_matrix:
    """DF(u) = [K] + T . a(u) + (T ._2 u) diag(a'(u)); Dirichlet rows -> identity,
    Dirichlet columns -> 0 (the reduced form of the block Jacobian of Sec. 4)."""
    J = contract_first(p.T, nodal_a(p, u)) + contract_mode2(p.T, u) @ sp.diags(nodal_da(p, u))
    if p.K is not None:
        J = J + p.K
    return _apply_dirichlet(p, J)


@dataclass
class NewtonStats:
    iterations: int = 0
    residual_norms: list = field(default_factory=list)
    status: str = "not_converged"
    backtracks: int = 0


def newton(p: Problem, u0: Optional[np.ndarray] = None, tol: float = 1e-10,
           max_iter: int = 50, residual_fn=None, jacobian_fn=None):
    """Damped Newton on F(u) = 0.  Stops when ||F|| <= tol ||F(u0)||.  A step is
    accepted when ||F(u + alpha delta)|| <= (1 - 1e-4 alpha) ||F(u)||, halving
    alpha up to 10 times; when no trial passes, the iteration stops with status
    'stagnated' (the residual has reached its rounding floor or the direction
    is no descent direction)."""
    residual_fn = residual_fn or (lambda v: residual(p, v))
    jacobian_fn = jacobian_fn or (lambda v: jacobian(p, v))
    u = np.zeros(p.n) if u0 is None else np.array(u0, dtype=np.float64)
    u[p.dirichlet] = 0.0
    F = residual_fn(u)
    nF = float(np.linalg.norm(F))
    nF0 = nF
    st = NewtonStats(residual_norms=[nF])
    if nF0 == 0.0:
        st.status = "converged"
        return u, st
    for it in range(max_iter):
        if nF <= tol * nF0:
            st.status = "converged"
            return u, st
        J = jacobian_fn(u)
        delta = spla.spsolve(J.tocsc(), -F)
        alpha = 1.0
        accepted = False
        for _ in range(11):
            ut = u + alpha * delta
            Ft = residual_fn(ut)
            nFt = float(np.linalg.norm(Ft))
            if np.isfinite(nFt) and nFt <= (1.0 - 1e-4 * alpha) * nF:
                accepted = True
                break
            alpha *= 0.5
            st.backtracks += 1
        if not accepted:
            st.status = "stagnated"
            return u, st
        u, F, nF = ut, Ft, nFt
        st.iterations = it + 1
        st.residual_norms.append(nF)
    st.status = "converged" if nF <= tol * nF0 else "not_converged"
    return u, st


# ----------------------------------------------------------------------------
# Picard iteration (Sec. 4, Example picard_iteration)
# ----------------------------------------------------------------------------
def picard_matrix(p: Problem, u: np.ndarray) -> sp.csr_matrix:
    """A(u) = [K] + T . a(u): the previous iterate substituted into the
    nonlinear coefficient, Dirichlet rows -> identity, columns -> 0."""
    A = contract_first(p.T, nodal_a(p, u))
    if p.K is not None:
        A = A + p.K
    return _apply_dirichlet(p, A)


@dataclass
class PicardStats:
    iterations: int = 0
    updates: list = field(default_factory=list)   # ||u^{n+1} - u^n|| / ||u^{n+1}||
    status: str = "not_converged"


def picard(p: Problem, u0: Optional[np.ndarray] = None, tol: float = 1e-12, max_iter: int = 500):
    """u^{n+1} = A(u^n)^{-1} d with d's Dirichlet rows zero (u_D = 0), the new
    coefficient a^{n+1} = a0 + (u^{n+1})^2 evaluated pointwise.  Stops when
    ||u^{n+1} - u^n||_2 <= tol ||u^{n+1}||_2."""
    u = np.zeros(p.n) if u0 is None else np.array(u0, dtype=np.float64)
    u[p.dirichlet] = 0.0
    b = p.d.copy()
    b[p.dirichlet] = 0.0
    st = PicardStats()
    for it in range(max_iter):
        un = spla.spsolve(picard_matrix(p, u).tocsc(), b)
        nu = float(np.linalg.norm(un))
        upd = float(np.linalg.norm(un - u)) / nu if nu > 0 else 0.0
        u = un
        st.iterations = it + 1
        st.updates.append(upd)
        if not np.isfinite(upd):
            st.status = "nonfinite"
            return u, st
        if upd <= tol:
            st.status = "converged"
            return u, st
    return u, st


# ----------------------------------------------------------------------------
# lifted EGFEM Newton on z = (u, a) exactly as in Sec. 4 (dense; tiny meshes)
# ----------------------------------------------------------------------------
def newton_lifted(p: Problem, tol: float = 1e-13, max_iter: int = 50):
    """z = (u, a);  F~(z) = [ [K u] + T:(u (x) a) - d ;  a - (a0 + u*u) ],
    D F~ = [[ [K] + T . a , T ._2 u ], [ -diag(2u), I ]] with the u-block's
    Dirichlet rows replaced by identity rows.  Full Newton steps."""
    n = p.n
    D = p.T.dense()
    Kd = p.K.toarray() if p.K is not None else np.zeros((n, n))
    u = np.zeros(n)
    a = p.a0 + u * u
    free = p.free

    def Ft(u, a):
        r1 = np.einsum("ijk,j,k->i", D, u, a) + Kd @ u - p.d
        r1[~free] = u[~free]
        r2 = a - (p.a0 + u * u)
        return np.concatenate([r1, r2])

    F = Ft(u, a)
    nF0 = np.linalg.norm(F)
    hist = [nF0]
    for _ in range(max_iter):
        if np.linalg.norm(F) <= tol * nF0:
            break
        Juu = np.einsum("ijk,k->ij", D, a) + Kd
        Jua = np.einsum("ijk,j->ik", D, u)
        Juu[~free, :] = 0.0
        Jua[~free, :] = 0.0
        Juu[~free, ~free] = 1.0
        Jau = -np.diag(2.0 * u)
        Jaa = np.eye(n)
        Jz = np.block([[Juu, Jua], [Jau, Jaa]])
        dz = np.linalg.solve(Jz, -F)
        u = u + dz[:n]
        a = a + dz[n:]
        F = Ft(u, a)
        hist.append(np.linalg.norm(F))
    return u, a, hist


# ----------------------------------------------------------------------------
# standard Galerkin approach (eq. nonlinear_terms / SGA_root), re-assembled
# by quadrature at every Newton iteration
# ----------------------------------------------------------------------------
def _sga_degree(form: int, dim: int) -> int:
    if dim == 1:
        return 5          # 3-point Gauss-Legendre
    return 2 if form == FORM_STIFF else 4


def sga_residual(p: Problem, u: np.ndarray, degree: Optional[int] = None) -> np.ndarray:
    """F_i = int (a0_h + u_h^2) grad u_h . grad phi_i - d_i           (stiffness)
       F_i = [K u]_i + int (a0_h + u_h^2) u_h phi_i - d_i            (mass form),
    with u_h, a0_h the P1 interpolants; exact-degree quadrature per element."""
    coords, cells = p.coords, p.cells
    dim = coords.shape[1]
    degree = degree or _sga_degree(p.form, dim)
    det, G = element_geometry(coords, cells)
    pts, wts = simplex_quadrature(dim, degree)
    lam = barycentric(pts)
    ue = u[cells]
    uq = ue @ lam.T                                  # [E, Q]
    aq = p.a0[cells] @ lam.T
    wq = det[:, None] * wts[None, :]
    if p.form == FORM_STIFF:
        gu = np.einsum("ea,ead->ed", ue, G)
        c = np.sum(wq * (aq + uq * uq), axis=1)
        Re = c[:, None] * np.einsum("ead,ed->ea", G, gu)
    else:
        Re = np.einsum("eq,qa->ea", wq * (aq + uq * uq) * uq, lam)
    F = np.bincount(cells.ravel(), weights=Re.ravel(), minlength=p.n) - p.d
    if p.K is not None:
        F = F + p.K @ u
    F[p.dirichlet] = 0.0
    return F


def sga_jacobian(p: Problem, u: np.ndarray, degree: Optional[int] = None) -> sp.csr_matrix:
    """D_u F re-assembled by quadrature (Sec. 4, Newton for the SGA)."""
    coords, cells = p.coords, p.cells
    dim = coords.shape[1]
    degree = degree or _sga_degree(p.form, dim)
    det, G = element_geometry(coords, cells)
    pts, wts = simplex_quadrature(dim, degree)
    lam = barycentric(pts)
    ue = u[cells]
    uq = ue @ lam.T
    aq = p.a0[cells] @ lam.T
    wq = det[:, None] * wts[None, :]
    if p.form == FORM_STIFF:
        gu = np.einsum("ea,ead->ed", ue, G)
        GG = np.einsum("ead,ebd->eab", G, G)
        c = np.sum(wq * (aq + uq * uq), axis=1)
        Gg = np.einsum("ead,ed->ea", G, gu)          # grad phi_a . grad u_h
        cross = np.einsum("eq,qb->eb", wq * 2.0 * uq, lam)   # int 2 u_h phi_b
        Je = c[:, None, None] * GG + Gg[:, :, None] * cross[:, None, :]
    else:
        Je = np.einsum("eq,qa,qb->eab", wq * (aq + 3.0 * uq * uq), lam, lam)
    J = _scatter_matrix(p.n, cells, Je)
    if p.K is not None:
        J = J + p.K
    return _apply_dirichlet(p, J)


def sga_newton(p: Problem, u0=None, tol: float = 1e-10, max_iter: int = 50):
    return newton(p, u0, tol, max_iter, residual_fn=lambda v: sga_residual(p, v),
                  jacobian_fn=lambda v: sga_jacobian(p, v))


# ----------------------------------------------------------------------------
# EGFEM with W_h = P2 (Case 1, exact reformulation of u^2), any dimension
# ----------------------------------------------------------------------------
@dataclass
class P2Space:
    n_u: int
    n_w: int
    edges: np.ndarray          # [n_edges, 2] global vertex pairs
    cell_dofs: np.ndarray      # [E, nl + n_local_edges] W-dof ids per element
    local_edges: list          # list of (a, b) local vertex pairs
    Pi: sp.csr_matrix          # interpolation Pi_u: V_h -> W_h dofs (Sec. 3.2)


def p2_space(coords, cells) -> P2Space:
    """P2 Lagrange dofs = vertices + edge midpoints; (Pi_u)_kj = phi_j(x_k)."""
    n = coords.shape[0]
    nl = cells.shape[1]
    local_edges = [(a, b) for a in range(nl) for b in range(a + 1, nl)]
    pairs = np.stack([np.sort(cells[:, [a, b]], axis=1) for (a, b) in local_edges], axis=1)
    flat = pairs.reshape(-1, 2).astype(np.int64)
    keys = flat[:, 0] * n + flat[:, 1]
    ukeys, inv = np.unique(keys, return_inverse=True)
    edges = np.stack([ukeys // n, ukeys % n], axis=1)
    edge_dof = n + inv.reshape(cells.shape[0], len(local_edges))
    cell_dofs = np.concatenate([cells.astype(np.int64), edge_dof], axis=1)
    ne = edges.shape[0]
    rows = np.concatenate([np.arange(n), n + np.arange(ne), n + np.arange(ne)])
    cols = np.concatenate([np.arange(n), edges[:, 0], edges[:, 1]])
    vals = np.concatenate([np.ones(n), 0.5 * np.ones(ne), 0.5 * np.ones(ne)])
    Pi = sp.coo_matrix((vals, (rows, cols)), shape=(n + ne, n)).tocsr()
    return P2Space(n, n + ne, edges, cell_dofs, local_edges, Pi)


def _p2_basis(lam: np.ndarray, local_edges) -> np.ndarray:
    """P2 nodal basis at points: vertex a -> lambda_a (2 lambda_a - 1),
    edge (a,b) -> 4 lambda_a lambda_b.  Returns [Q, nl + n_edges]."""
    vert = lam * (2.0 * lam - 1.0)
    edge = np.stack([4.0 * lam[:, a] * lam[:, b] for (a, b) in local_edges], axis=1)
    return np.concatenate([vert, edge], axis=1)


def assemble_tensor_p2(coords, cells, W: P2Space, form: int):
    """T_ijk = int eta_k grad phi_j . grad phi_i (or eta_k phi_j phi_i, or
    eta_k phi_j sum_d d_d phi_i for the convection form) with eta the P2 basis of
    W_h; returned as COO arrays with k over W-dofs."""
    dim = coords.shape[1]
    det, G = element_geometry(coords, cells)
    pts, wts = simplex_quadrature(dim, {FORM_STIFF: 2, FORM_MASS: 4, FORM_CONV: 3}[form])
    lam = barycentric(pts)
    eta = _p2_basis(lam, W.local_edges)
    nl = dim + 1
    nw = eta.shape[1]
    if form == FORM_STIFF:
        GG = np.einsum("ead,ebd->eab", G, G)
        psi = np.einsum("q,qc->c", wts, eta)
        Te = det[:, None, None, None] * GG[:, :, :, None] * psi[None, None, None, :]
    elif form == FORM_CONV:
        gsum = G.sum(axis=2)
        gsum[np.abs(gsum) <= 1e-12 * np.abs(G).sum(axis=2)] = 0.0
        pair = np.einsum("q,qb,qc->bc", wts, lam, eta)             # int phi_b eta_c on the reference
        Te = det[:, None, None, None] * gsum[:, :, None, None] * pair[None, None]
    else:
        trip = np.einsum("q,qa,qb,qc->abc", wts, lam, lam, eta)
        Te = det[:, None, None, None] * trip[None]
    ai, bi, ci = np.meshgrid(np.arange(nl), np.arange(nl), np.arange(nw), indexing="ij")
    I = cells[:, ai.ravel()].ravel().astype(np.int64)
    J = cells[:, bi.ravel()].ravel().astype(np.int64)
    K = W.cell_dofs[:, ci.ravel()].ravel()
    return I, J, K, Te.reshape(-1)


def tensor_p2(coords, cells, form: int, drop_rel: float = DROP_REL):
    """The P2 tensor with duplicates summed and the exact-zero drop rule applied
    (as for the P1 tensors); the returned Tensor3 has n = n_w, rows and j below
    the vertex count, k over all P2 dofs (vertices, then edges in ascending
    (min, max) vertex order).  Returns (tensor, space)."""
    W = p2_space(coords, cells)
    I, J, K, V = assemble_tensor_p2(coords, cells, W, form)
    return _merge_coo3(W.n_w, I, J, K, V, drop_rel), W


@dataclass
class ProblemP2:
    base: Problem
    W: P2Space
    I: np.ndarray
    J: np.ndarray
    K: np.ndarray
    V: np.ndarray


def build_problem_p2(p: Problem) -> ProblemP2:
    W = p2_space(p.coords, p.cells)
    I, J, K, V = assemble_tensor_p2(p.coords, p.cells, W, p.form)
    return ProblemP2(p, W, I, J, K, V)


def residual_p2(q: ProblemP2, u: np.ndarray) -> np.ndarray:
    """F = [K u] + T^{P2}:(u (x) a_W) - d with a_W = Pi a0 + (Pi u)^2 at the P2 dofs."""
    p = q.base
    Pu = q.W.Pi @ u
    aW = q.W.Pi @ p.a0 + Pu * Pu
    F = np.bincount(q.I, weights=q.V * u[q.J] * aW[q.K], minlength=p.n) - p.d
    if p.K is not None:
        F = F + p.K @ u
    F[p.dirichlet] = 0.0
    return F


def jacobian_p2(q: ProblemP2, u: np.ndarray) -> sp.csr_matrix:
    p = q.base
    Pu = q.W.Pi @ u
    aW = q.W.Pi @ p.a0 + Pu * Pu
    n, nw = p.n, q.W.n_w
    A = sp.coo_matrix((q.V * aW[q.K], (q.I, q.J)), shape=(n, n)).tocsr()
    B = sp.coo_matrix((q.V * u[q.J], (q.I, q.K)), shape=(n, nw)).tocsr()
    J = A + B @ sp.diags(2.0 * Pu) @ q.W.Pi
    if p.K is not None:
        J = J + p.K
    return _apply_dirichlet(p, J.tocsr())


def newton_p2(q: ProblemP2, tol=1e-13, max_iter=50):
    return newton(q.base, None, tol, max_iter, residual_fn=lambda v: residual_p2(q, v),
                  jacobian_fn=lambda v: jacobian_p2(q, v))


# ----------------------------------------------------------------------------
# EGFEM with W_h = I_k, the quadrature-point space (Case 3 of Sec. 3.1)
# ----------------------------------------------------------------------------
def iq_rule(dim: int):
    """The fixed quadrature rule whose points carry the coefficient: barycentric
    points [Q, dim+1] and weights [Q] relative to |e|.
      1D: 2-point Gauss-Legendre, x = 1/2 -+ 1/(2 sqrt 3), weights 1/2 (degree 3);
      2D: the 3 interior points with barycentrics (2/3, 1/6, 1/6) and permutations,
          weights 1/3 (degree 2);
      3D: the 4 points with barycentrics (a, b, b, b) and permutations,
          a = (5 + 3 sqrt 5) / 20, b = (5 - sqrt 5) / 20, weights 1/4 (degree 2)."""
    if dim == 1:
        x = 0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0)
        lam = np.array([[1.0 - x[0], x[0]], [1.0 - x[1], x[1]]])
        return lam, np.array([0.5, 0.5])
    if dim == 2:
        lam = np.full((3, 3), 1.0 / 6.0)
        np.fill_diagonal(lam, 2.0 / 3.0)
        return lam, np.full(3, 1.0 / 3.0)
    a = (5.0 + 3.0 * math.sqrt(5.0)) / 20.0
    b = (5.0 - math.sqrt(5.0)) / 20.0
    lam = np.full((4, 4), b)
    np.fill_diagonal(lam, a)
    return lam, np.full(4, 0.25)


@dataclass
class IQSpace:
    n_u: int
    n_w: int                   # cells * points: dof k = e * Q + q
    lam: np.ndarray            # [Q, d+1] barycentrics of the points
    wts: np.ndarray            # [Q] weights relative to |e|
    Pi: sp.csr_matrix          # (Pi_u)_kj = phi_j(x_k): evaluation of the P1 function at the points


def iq_space(coords, cells) -> IQSpace:
    n = coords.shape[0]
    dim = coords.shape[1]
    lam, wts = iq_rule(dim)
    E, Q, nl = cells.shape[0], lam.shape[0], dim + 1
    rows = np.repeat(np.arange(E * Q), nl)
    cols = np.repeat(cells, Q, axis=0).ravel()
    vals = np.tile(lam.ravel(), E)
    Pi = sp.coo_matrix((vals, (rows, cols)), shape=(E * Q, n)).tocsr()
    return IQSpace(n, E * Q, lam, wts, Pi)


def tensor_iq(coords, cells, form: int, drop_rel: float = DROP_REL):
    """T_ijk = w_q |e| grad phi_j . grad phi_i (x_q)       (stiffness),
    T_ijk = w_q |e| phi_j(x_q) phi_i(x_q)                   (mass), or
    T_ijk = w_q |e| phi_j(x_q) sum_d d_d phi_i              (convection, Sec. 5.2), k = (e, q):
    the trilinear forms with eta_k the quadrature functional at x_q.  Returns
    (tensor with n = n_w, space)."""
    W = iq_space(coords, cells)
    dim = coords.shape[1]
    det, G = element_geometry(coords, cells)
    vol = det / math.factorial(dim)
    nl, Q = dim + 1, W.lam.shape[0]
    if form == FORM_STIFF:
        GG = np.einsum("ead,ebd->eab", G, G)
        Te = vol[:, None, None, None] * GG[:, :, :, None] * W.wts[None, None, None, :]
    elif form == FORM_MASS:
        LL = np.einsum("q,qa,qb->abq", W.wts, W.lam, W.lam)
        Te = vol[:, None, None, None] * LL[None]
    elif form == FORM_CONV:
        gsum = G.sum(axis=2)                                 # sum_d d_d phi_a, [E, d+1]
        gsum[np.abs(gsum) <= 1e-12 * np.abs(G).sum(axis=2)] = 0.0
        LW = np.einsum("q,qb->bq", W.wts, W.lam)             # w_q phi_b(x_q)
        Te = vol[:, None, None, None] * gsum[:, :, None, None] * LW[None, None]
    else:
        raise ValueError("unknown form")
    ai, bi, qi = np.meshgrid(np.arange(nl), np.arange(nl), np.arange(Q), indexing="ij")
    E = cells.shape[0]
    I = cells[:, ai.ravel()].ravel().astype(np.int64)
    J = cells[:, bi.ravel()].ravel().astype(np.int64)
    K = (np.arange(E)[:, None] * Q + qi.ravel()[None, :]).ravel().astype(np.int64)
    return _merge_coo3(W.n_w, I, J, K, Te.reshape(-1), drop_rel), W


def build_problem_iq(p: Problem) -> ProblemP2:
    """The problem with the coefficient on I_k: residual_p2 / jacobian_p2 /
    newton_p2 apply unchanged (they use only Pi and the tensor)."""
    T, W = tensor_iq(p.coords, p.cells, p.form)
    return ProblemP2(p, W, T.i, T.j, T.k, T.v)


# ----------------------------------------------------------------------------
# EGFEM with W_h = P0 and the gradient interpolation (Sec. 3.2; the p-Laplace and
# minimal surface examples of Sec. 5): a(grad u) = (c0 + c1 |grad u|^2)^q
# ----------------------------------------------------------------------------
@dataclass
class GradProblem:
    n: int
    coords: np.ndarray
    cells: np.ndarray
    T: Tensor3                 # T_ijk = int eta_k grad phi_j . grad phi_i = K^{e_k}_ij (k = cell)
    d: np.ndarray              # load M f
    dirichlet: np.ndarray      # bool
    c0: float
    c1: float
    q: float

    @property
    def free(self) -> np.ndarray:
        return ~self.dirichlet


def tensor_p0(coords, cells, drop_rel: float = DROP_REL) -> Tensor3:
    """eta_k the indicator of cell k, so T_ijk = |e_k| grad phi_j . grad phi_i on e_k;
    the returned Tensor3 has n = max(nodes, cells) (k indexes cells)."""
    det, G = element_geometry(coords, cells)
    dim = coords.shape[1]
    vol = det / math.factorial(dim)
    Ke = vol[:, None, None] * np.einsum("ead,ebd->eab", G, G)
    nl = dim + 1
    E = cells.shape[0]
    ai, bi = np.meshgrid(np.arange(nl), np.arange(nl), indexing="ij")
    I = cells[:, ai.ravel()].ravel().astype(np.int64)
    J = cells[:, bi.ravel()].ravel().astype(np.int64)
    K = np.repeat(np.arange(E, dtype=np.int64), nl * nl)
    return _merge_coo3(max(coords.shape[0], E), I, J, K, Ke.reshape(-1), drop_rel)


def build_grad_problem(workload) -> GradProblem:
    m = workload.mesh
    M = assemble_mass(m.coords, m.cells)
    return GradProblem(m.n_nodes, m.coords, m.cells, tensor_p0(m.coords, m.cells), M @ workload.f,
                       m.dirichlet.astype(bool), workload.c0, workload.c1, workload.q)


def grad_interp(p: GradProblem, u: np.ndarray) -> np.ndarray:
    """Pi_grad u: the (constant) gradient of u_h on every cell, [cells, dim]."""
    _, G = element_geometry(p.coords, p.cells)
    return np.einsum("ea,ead->ed", u[p.cells], G)


def grad_coef(p: GradProblem, u: np.ndarray) -> np.ndarray:
    """a_e = (c0 + c1 |grad u_h|_e|^2)^q, the nonlinearity at the P0 dofs (+inf
    where the base is 0 and q < 0)."""
    z = grad_interp(p, u)
    with np.errstate(divide="ignore"):
        return (p.c0 + p.c1 * np.sum(z * z, axis=1)) ** p.q


def grad_matrix(p: GradProblem, a: np.ndarray) -> sp.csr_matrix:
    """(T . a)_ij = sum_e a_e K^e_ij with Dirichlet identity rows and zero columns.
    Only entries with a free row and a free column are formed: a cell whose
    vertices all lie on the boundary has u_h = 0, grad u_h = 0 and, for q < 0 and
    c0 = 0, an unbounded coefficient, but it couples Dirichlet nodes only."""
    T = p.T
    keep = p.free[T.i] & p.free[T.j]
    A = sp.coo_matrix((T.v[keep] * a[T.k[keep]], (T.i[keep], T.j[keep])), shape=(p.n, p.n)).tocsr()
    return (A + sp.diags(p.dirichlet.astype(np.float64))).tocsr()


def residual_grad(p: GradProblem, u: np.ndarray) -> np.ndarray:
    """F = T:(u (x) a(grad u)) - d on the free rows (Dirichlet rows 0)."""
    a = grad_coef(p, u)
    T = p.T
    keep = p.free[T.i]
    F = np.bincount(T.i[keep], weights=T.v[keep] * u[T.j[keep]] * a[T.k[keep]], minlength=p.n) - p.d
    F[p.dirichlet] = 0.0
    return F


def picard_grad(p: GradProblem, u0: Optional[np.ndarray] = None, tol: float = 1e-12, max_iter: int = 500,
                start_linear: bool = True):
    """Picard iteration of the examples: (T . a^n) u^{n+1} = d, a^{n+1} = a(Pi_grad u^{n+1});
    with start_linear the first matrix uses a = 1 (a Laplace solve), which also
    serves p < 2 where a(0) is unbounded.  Exact solves; stops on the relative
    update.  Returns (u, iterations)."""
    u = np.zeros(p.n) if u0 is None else np.array(u0, dtype=np.float64)
    u[p.dirichlet] = 0.0
    rhs = p.d.copy()
    rhs[p.dirichlet] = 0.0
    for it in range(max_iter):
        a = np.ones(p.cells.shape[0]) if (it == 0 and start_linear) else grad_coef(p, u)
        un = spla.spsolve(grad_matrix(p, a).tocsc(), rhs)
        upd = np.linalg.norm(un - u) / max(np.linalg.norm(un), 1e-300)
        u = un
        if upd <= tol:
            return u, it + 1
    return u, max_iter


def jacobian_grad(p: GradProblem, u: np.ndarray) -> sp.csr_matrix:
    """DF(u) for F = T:(u (x) a(grad u)) - d with a_e = (c0 + c1 |z_e|^2)^q, z_e = grad u_h|_e:
    the product rule gives, per cell, a_e K^e plus the derivative of a_e,
    d a_e / d u_j = a'_e z_e . grad lambda_j with a'_e = 2 q c1 (c0 + c1 |z_e|^2)^(q-1),
    times (K^e u_e)_i = |e| grad lambda_i . z_e.  Free rows and columns only;
    Dirichlet rows identity."""
    det, G = element_geometry(p.coords, p.cells)
    dim = p.coords.shape[1]
    vol = det / math.factorial(dim)
    z = np.einsum("ea,ead->ed", u[p.cells], G)
    base = p.c0 + p.c1 * np.sum(z * z, axis=1)
    keep = p.free[p.cells].any(axis=1)          # cells with a free vertex
    with np.errstate(divide="ignore", invalid="ignore"):
        a = np.where(keep, base, 1.0) ** p.q
        ap = 2.0 * p.q * p.c1 * np.where(keep, base, 1.0) ** (p.q - 1.0)
    GG = np.einsum("ead,ebd->eab", G, G)
    gz = np.einsum("ead,ed->ea", G, z)
    Je = vol[:, None, None] * (a[:, None, None] * GG + ap[:, None, None] * gz[:, :, None] * gz[:, None, :])
    nl = dim + 1
    rows = np.repeat(p.cells, nl, axis=1).ravel()
    cols = np.tile(p.cells, (1, nl)).ravel()
    vals = Je.reshape(-1)
    m = p.free[rows] & p.free[cols]
    J = sp.coo_matrix((vals[m], (rows[m], cols[m])), shape=(p.n, p.n)).tocsr()
    return (J + sp.diags(p.dirichlet.astype(np.float64))).tocsr()


def newton_grad(p: GradProblem, tol: float = 1e-10, max_iter: int = 50):
    """Damped Newton (the rule of `newton`) for the gradient nonlinearity,
    started from the Laplace solution (the first Picard step with a = 1).
    Returns (u, NewtonStats)."""
    u0, _ = picard_grad(p, tol=0.0, max_iter=1)
    return newton(p, u0, tol, max_iter, residual_fn=lambda v: residual_grad(p, v),
                  jacobian_fn=lambda v: jacobian_grad(p, v))


# ----------------------------------------------------------------------------
# adjoint of the converged solve (implicit function theorem)
# ----------------------------------------------------------------------------
def adjoint_gradients(p: Problem, u_star: np.ndarray, ubar: np.ndarray):
    """For an objective with dJ/du = ubar at the solution u* of F(u; d(f), a0) = 0:
       J(u*)^T lam = ubar (free rows; lam_D = 0),
       dJ/df   = M lam               (F depends on f through -d = -M f),
       dJ/da0  = -(T ._2 u*)^T lam,  i.e. -sum_ij lam_i T_ijk u*_j.
    Returns (lam, grad_f, grad_a0)."""
    J = jacobian(p, u_star)
    rhs = np.array(ubar, dtype=np.float64)
    rhs[p.dirichlet] = 0.0
    lam = spla.spsolve(J.T.tocsc(), rhs)
    grad_f = p.M @ lam
    grad_a0 = -contract_mode3(p.T, lam, u_star)
    return lam, grad_f, grad_a0


def tracking_objective(u: np.ndarray, u_d: np.ndarray) -> float:
    """J = 0.5 sum_i (u_i - u_d,i)^2 (nodal Euclidean)."""
    r = u - u_d
    return 0.5 * float(r @ r)


# ----------------------------------------------------------------------------
# the stream sizes of the stored tensor, for byte accounting
# ----------------------------------------------------------------------------
# ----------------------------------------------------------------------------
# viscous Burgers' equation, semi-implicit time stepping (Sec. 5.2)
# ----------------------------------------------------------------------------
@dataclass
class BurgersSystem:
    N: Tensor3                  # convection tensor N_ijk = int phi_k phi_j (d_1 + d_2) phi_i
    Nf: sp.csr_matrix           # group matrix N^f_ik = int phi_k (d_1 + d_2) phi_i = sum_j N_ijk
    M: sp.csr_matrix
    K: sp.csr_matrix
    S: sp.csr_matrix            # M + dt nu K, Dirichlet rows identity, Dirichlet columns 0
    free: np.ndarray            # bool [N]
    dt: float
    nu: float


def burgers_system(coords, cells, dirichlet, dt: float, nu: float) -> BurgersSystem:
    """The offline part of the semi-implicit scheme: N (tensor formulation), N^f
    (group formulation with W_h = V_h = P1, where interpolating u^2 gives
    N^f (u . u) and N^f = N contracted with the constant 1 in j, by the partition
    of unity), M, K and the constant system matrix M + dt nu K."""
    N = assemble_tensor(coords, cells, FORM_CONV)
    Nf = contract_mode2(N, np.ones(N.n))
    M = assemble_mass(coords, cells)
    K = assemble_stiffness(coords, cells)
    free = np.asarray(dirichlet) == 0
    S = (M + (dt * nu) * K).tocsr()
    Df = sp.diags(free.astype(np.float64))
    S = (Df @ S @ Df + sp.diags((~free).astype(np.float64))).tocsr()
    return BurgersSystem(N, Nf, M, K, S, free, dt, nu)


def burgers_group_p2(coords, cells):
    """EGFEM group matrix with W_h = P2 (Sec. 5.2): N^f_ik = int eta_k sum_d d_d phi_i
    for the P2 basis eta, i.e. the P2 convection tensor summed over j (partition
    of unity), with f = (Pi_u u)^2 at the P2 dofs.  Returns (N^f [n, n_w], space)."""
    T, W = tensor_p2(coords, cells, FORM_CONV)
    n = coords.shape[0]
    Nf = sp.coo_matrix((T.v, (T.i, T.k)), shape=(n, W.n_w)).tocsr()
    return Nf, W


def burgers_group_iq(coords, cells):
    """EGFEM group matrix with W_h = I_k (the quadrature-point space; Sec. 5.2
    compares EGFEM(I_3)): N^f_ik = w_q |e| sum_d d_d phi_i for k = (e, q), the I_k
    convection tensor summed over j (partition of unity), with f = (Pi_u u)^2
    at the points.  Returns (N^f [n, n_w], space); burgers() takes it as
    group_p2 (any (N^f, space) pair with the space's Pi)."""
    T, W = tensor_iq(coords, cells, FORM_CONV)
    n = coords.shape[0]
    Nf = sp.coo_matrix((T.v, (T.i, T.k)), shape=(n, W.n_w)).tocsr()
    return Nf, W


def burgers(sysm: BurgersSystem, u0: np.ndarray, source: Optional[np.ndarray], steps: int,
            group: bool = False, history: bool = False, group_p2=None):
    """Semi-implicit Euler steps of Sec. 5.2,
        M (u^{n+1} - u^n) + dt (nu K u^{n+1} - 1/2 C(u^n) - d^{n+1}) = 0,
    i.e. (M + dt nu K) u^{n+1} = M u^n + dt (1/2 C(u^n) + d^{n+1}), with
        C(u) = N : (u (x) u)       (tensor formulation, exact for P1 u), or
        C(u) = N^f (u . u)         (group formulation: u^2 interpolated onto P1),
    load d^{n+1} = M s^{n+1} for the nodal source values s^{n+1} = source[n]
    (source None: no source), zero Dirichlet data; with group_p2 = (N^f, space)
    from burgers_group_p2 (or burgers_group_iq) the group formulation uses
    W_h = P2 (or I_k) instead.  Each
    linear system is solved directly (one LU factorisation of the constant
    matrix).  Returns u^steps, or the list [u^0, ..., u^steps] with history=True."""
    u = np.array(u0, dtype=np.float64, copy=True)
    u[~sysm.free] = 0.0
    lu = spla.splu(sysm.S.tocsc())
    out = [u.copy()] if history else None
    for n in range(steps):
        if group_p2 is not None:
            # EGFEM with W_h = P2 (or I_k): f = (Pi_u u)^2 at the dofs of W_h
            Nf2, W2 = group_p2
            pu = W2.Pi @ u
            conv = Nf2 @ (pu * pu)
        else:
            conv = sysm.Nf @ (u * u) if group else contract_uv(sysm.N, u, u)
        x = u if source is None else u + sysm.dt * source[n]
        rhs = sysm.M @ x + (0.5 * sysm.dt) * conv
        rhs[~sysm.free] = 0.0
        u = lu.solve(rhs)
        if history:
            out.append(u.copy())
    return out if history else u


def slot_count(T: Tensor3) -> int:
    """Number of distinct (i, j) pairs carrying at least one stored T_ijk."""
    return int(np.unique(T.i * T.n + T.j).size)
