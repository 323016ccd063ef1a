"""Gradient nonlinearities with W_h = P0 on the GPU against the oracle: the
tensor T_ijk = K^{e_k}_ij, the action and emission with a coefficient per cell,
and the Picard iteration of the p-Laplace and minimal-surface examples."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import workloads as W
from oracle import egfem_oracle as O
from test_gpu_parity import DEV, csr_of, dt, eg, host, irregular_mesh, relerr

pytestmark = pytest.mark.gpu

MESHES = {
    "1d_n24": lambda: W.mesh_1d(24),
    "2d_n9": lambda: W.mesh_2d(9),
    "disk_n12": lambda: W.mesh_disk(12),
    "2d_jitter_n15": lambda: irregular_mesh(15),
    "3d_n4": lambda: W.mesh_3d(4),
}


def _p0(m, form=0):
    print(f"p0 build dim={m.dim} n={m.n} form={form}", flush=True)
    return eg().Tensor.from_mesh(m, form, wspace=eg().W_P0)


@pytest.mark.parametrize("mesh", list(MESHES))
def test_p0_tensor_action_and_emission(mesh):
    m = MESHES[mesh]()
    T = _p0(m)
    To = O.tensor_p0(m.coords, m.cells)
    E, n = m.n_cells, m.n_nodes
    assert T.info.wspace == 3 and T.info.n_w == E and T.info.nnz == To.nnz
    i, j, k, v = T.export()
    kg = (i.astype(np.int64) * n + j) * E + k
    ko = (To.i * n + To.j) * E + To.k
    og, oo = np.argsort(kg), np.argsort(ko)
    assert np.array_equal(kg[og], ko[oo])
    assert np.abs(v[og] - To.v[oo]).max() <= 1e-14 * np.abs(To.v).max()
    rng = np.random.default_rng(51)
    u = rng.uniform(-1, 1, n)
    a = rng.uniform(0.5, 2, E)
    r = host(T.residual(dt(u), dt(a)))
    ro = np.bincount(To.i, weights=To.v * u[To.j] * a[To.k], minlength=max(n, E))[:n]
    assert relerr(r, ro) < 1e-12
    dirm = m.dirichlet.astype(bool)
    Jg = csr_of(T, T.jacobian(dt(u), dt(a), dirichlet=dt(m.dirichlet, torch.uint8)))
    A = sp.coo_matrix((To.v * a[To.k], (To.i, To.j)), shape=(n, n)).tocsr()
    f = sp.diags((~dirm).astype(float))
    Jo = (f @ A @ f + sp.diags(dirm.astype(float))).tocsr()
    assert abs(Jg - Jo).max() <= 1e-12 * abs(Jo).max()
    # the mass form: T . 1 is the mass matrix
    Tm = _p0(m, 1)
    Jm = csr_of(Tm, Tm.jacobian(dt(u), dt(np.ones(E))))
    Mo = O.assemble_mass(m.coords, m.cells)
    assert abs(Jm - Mo).max() <= 1e-14 * abs(Mo).max()


def _load(T, m, f):
    return T.matvec(dt(f), "M")


CASES = {
    # name: (mesh, source, c0, c1, q)
    "plaplace_1d_p1.5": (lambda: W.mesh_1d(64), 1.0, 0.0, 1.0, -0.25),
    "plaplace_disk_n16_p1.5": (lambda: W.mesh_disk(16), 1.0, 0.0, 1.0, -0.25),
    "minimal_surface_n20": (lambda: W.mesh_2d(20), 1.0, 1.0, 1.0, -0.5),
    "plaplace_3d_n5_p1.8": (lambda: W.mesh_3d(5), 1.0, 0.0, 1.0, -0.1),
}


@pytest.mark.parametrize("name", list(CASES))
def test_picard_grad_matches_oracle(name):
    mk, fval, c0, c1, q = CASES[name]
    m = mk()
    print(f"picard_grad {name}", flush=True)
    T = _p0(m)
    f = np.full(m.n_nodes, fval)
    p = eg().Problem(T.n, _load(T, m, f), dt(m.dirichlet, torch.uint8))
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st = T.picard_grad(p, u, c0, c1, q, opts=eg().PicardOptions(tol=1e-13, krylov_rtol=1e-6), warn=False)
    assert st.status == 0, st.status_name
    wl = W.GradientWorkload("t", m, f, 0.0, c0, c1, q, None)
    P = O.build_grad_problem(wl)
    uo, it = O.picard_grad(P, tol=1e-13)
    ug = host(u)
    assert relerr(ug, uo) <= 1e-10
    assert np.linalg.norm(O.residual_grad(P, ug)) <= 1e-10 * np.linalg.norm(P.d[P.free])
    assert st.res <= 1e-10 * np.linalg.norm(P.d[P.free])
    assert st.picard_iters <= it + 5


def test_picard_grad_full_size_disk():
    """The paper's p-Laplace example (p = 3/2, unit disk, source 1) at 66,049
    nodes: the oracle's fixed point and O(h^2) closeness to the radial solution."""
    wl = W.plaplace_disk(256)
    T = _p0(wl.mesh)
    p = eg().Problem(T.n, _load(T, wl.mesh, wl.f), dt(wl.mesh.dirichlet, torch.uint8))
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st = T.picard_grad(p, u, wl.c0, wl.c1, wl.q)
    assert st.status == 0
    P = O.build_grad_problem(wl)
    ug = host(u)
    assert np.linalg.norm(O.residual_grad(P, ug)) <= 1e-9 * np.linalg.norm(P.d[P.free])
    assert np.linalg.norm(ug - wl.exact) / np.linalg.norm(wl.exact) < 1e-4


def test_picard_grad_rejections_and_determinism():
    m = W.mesh_disk(10)
    T = _p0(m)
    p = eg().Problem(T.n, _load(T, m, np.ones(m.n_nodes)), dt(m.dirichlet, torch.uint8))
    u1 = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    u2 = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    T.picard_grad(p, u1, 0.0, 1.0, -0.25)
    T.picard_grad(p, u2, 0.0, 1.0, -0.25)
    assert torch.equal(u1, u2)
    with pytest.raises(eg().EgfemError):
        T.newton(p, u1)
    with pytest.raises(eg().EgfemError):
        T.picard(p, u1)
    with pytest.raises(eg().EgfemError):
        T.jacobian(u1, dt(np.ones(m.n_cells)), dt(np.ones(m.n_cells)))
    with pytest.raises(eg().EgfemError):
        T.picard_grad(p, u1, -1.0, 1.0, 0.5)
    S = eg().Tensor.from_mesh(m, 0)
    with pytest.raises(eg().EgfemError):
        S.picard_grad(p, u1, 0.0, 1.0, -0.25)


@pytest.mark.parametrize("name", list(CASES))
def test_newton_grad_matches_oracle(name):
    """Damped Newton with the analytic Jacobian (per-cell derivative weights in
    the W-slot emission) reaches the oracle's Newton solution, which is also the
    Picard fixed point."""
    mk, fval, c0, c1, q = CASES[name]
    m = mk()
    print(f"newton_grad {name}", flush=True)
    T = _p0(m)
    f = np.full(m.n_nodes, fval)
    p = eg().Problem(T.n, _load(T, m, f), dt(m.dirichlet, torch.uint8))
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    # tol 1e-12 lies above the rounding floor of ||F|| (~1e-13 ||F_0||), where
    # further steps only shuffle rounding noise
    st = T.newton_grad(p, u, c0, c1, q, opts=eg().NewtonOptions(tol=1e-12, krylov_rtol=1e-13), warn=False)
    assert st.status == 0, st.status_name
    wl = W.GradientWorkload("t", m, f, 0.0, c0, c1, q, None)
    P = O.build_grad_problem(wl)
    uo, sto = O.newton_grad(P, tol=1e-12)
    assert sto.status == "converged"
    ug = host(u)
    assert relerr(ug, uo) <= 1e-10
    assert np.linalg.norm(O.residual_grad(P, ug)) <= 1e-11 * np.linalg.norm(P.d[P.free])
    assert st.newton_iters <= sto.iterations + 2


def test_newton_grad_full_size_disk_and_forcing():
    wl = W.plaplace_disk(256)
    T = _p0(wl.mesh)
    p = eg().Problem(T.n, _load(T, wl.mesh, wl.f), dt(wl.mesh.dirichlet, torch.uint8))
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st = T.newton_grad(p, u, wl.c0, wl.c1, wl.q, opts=eg().NewtonOptions(tol=1e-10, forcing=1))
    # the step count follows the inexact (forcing-term) solves, which depend on
    # the Krylov grid and preconditioner: 9 to 14 steps have been seen
    assert st.status == 0 and st.newton_iters <= 16
    P = O.build_grad_problem(wl)
    ug = host(u)
    assert np.linalg.norm(O.residual_grad(P, ug)) <= 2e-10 * np.linalg.norm(P.d[P.free])
    assert np.linalg.norm(ug - wl.exact) / np.linalg.norm(wl.exact) < 1e-4
    # deterministic, and the Picard fixed point
    u2 = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    T.newton_grad(p, u2, wl.c0, wl.c1, wl.q, opts=eg().NewtonOptions(tol=1e-10, forcing=1))
    assert torch.equal(u, u2)
    up = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    T.picard_grad(p, up, wl.c0, wl.c1, wl.q)
    assert relerr(ug, host(up)) < 1e-8


def test_picard_grad_timing_leaves_the_iteration_unchanged():
    """With timing on, the gradient-coefficient Picard iteration gives bitwise
    the untimed iterate and statistics, and reports the CG time."""
    m = W.mesh_disk(16)
    T = _p0(m)
    p = eg().Problem(T.n, _load(T, m, np.ones(m.n_nodes)), dt(m.dirichlet, torch.uint8))
    runs = []
    for timing in (0, 1):
        u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
        st = T.picard_grad(p, u, 0.0, 1.0, -0.25, opts=eg().PicardOptions(timing=timing), warn=False)
        assert st.status == 0, st.status_name
        assert st.picard_iters <= 64 and sum(st.krylov_hist) == st.krylov_iters
        assert (st.t_krylov_ms > 0.0) == bool(timing)
        runs.append((u, st))
    (u0, s0), (u1, s1) = runs
    assert torch.equal(u0, u1)
    assert s0.picard_iters == s1.picard_iters and s0.krylov_hist == s1.krylov_hist
    assert s0.update_hist == s1.update_hist


def test_newton_grad_timing_leaves_the_iteration_unchanged():
    """With timing on, the gradient-coefficient Newton iteration gives bitwise
    the untimed iterate and statistics, and reports the Krylov time."""
    m = W.mesh_disk(16)
    T = _p0(m)
    p = eg().Problem(T.n, _load(T, m, np.ones(m.n_nodes)), dt(m.dirichlet, torch.uint8))
    runs = []
    for timing in (0, 1):
        u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
        st = T.newton_grad(p, u, 0.0, 1.0, -0.25, opts=eg().NewtonOptions(tol=1e-10, forcing=1, timing=timing),
                           warn=False)
        assert st.status == 0, st.status_name
        # the total also holds the Laplace start solve, the per-step counts do not
        assert st.newton_iters <= 64 and sum(st.krylov_hist) < st.krylov_iters
        assert (st.t_krylov_ms > 0.0) == bool(timing)
        runs.append((u, st))
    (u0, s0), (u1, s1) = runs
    assert torch.equal(u0, u1)
    assert s0.krylov_hist == s1.krylov_hist and s0.res_hist == s1.res_hist
    assert s0.krylov_iters == s1.krylov_iters
