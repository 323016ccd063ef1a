"""Coefficient spaces W_h != V_h on the GPU against the oracle: P2 (Case 1 of
Sec. 3.1) and the quadrature-point space I_k (Case 3).  The tensor entry by
entry, the raw action and Jacobian with coefficients on the dofs of W_h, the
problem residual / Jacobian with a = Pi a0 + (Pi u)^2, and Newton and Picard
solutions, which for the stiffness form also equal the standard Galerkin (SGA)
solution."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import workloads as W
from oracle import egfem_oracle as O
from test_gpu_parity import DEV, csr_of, dt, eg, gpu_problem, host, irregular_mesh, relerr

pytestmark = pytest.mark.gpu

MESHES = {
    "1d_n16": lambda: W.mesh_1d(16),
    "2d_n8": lambda: W.mesh_2d(8),
    "2d_n23": lambda: W.mesh_2d(23),
    "2d_jitter_n13": lambda: irregular_mesh(13),
    "3d_n2": lambda: W.mesh_3d(2),
    "3d_n5": lambda: W.mesh_3d(5),
}


SPACES = {
    "p2": (lambda: eg().W_P2, O.tensor_p2, O.build_problem_p2),
    "iq": (lambda: eg().W_IQ, O.tensor_iq, O.build_problem_iq),
}


def _p2(m, form, space="p2"):
    print(f"{space} build dim={m.dim} n={m.n} form={form}", flush=True)
    return eg().Tensor.from_mesh(m, form, wspace=SPACES[space][0]())


@pytest.mark.parametrize("space", list(SPACES))
@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("mesh", list(MESHES))
def test_p2_build_matches_oracle(mesh, form, space):
    m = MESHES[mesh]()
    T = _p2(m, form, space)
    To, Wsp = SPACES[space][1](m.coords, m.cells, form)
    assert T.info.wspace == SPACES[space][0]() and T.info.n_w == Wsp.n_w
    assert T.info.nnz == To.nnz and T.info.structural_nnz == To.structural_nnz
    i, j, k, v = T.export()
    nw = Wsp.n_w
    kg = (i.astype(np.int64) * nw + j) * nw + k
    ko = (To.i * nw + To.j) * nw + To.k
    og, oo = np.argsort(kg), np.argsort(ko)
    assert np.array_equal(kg[og], ko[oo])
    assert np.abs(v[og] - To.v[oo]).max() <= 1e-14 * np.abs(To.v).max()


@pytest.mark.parametrize("space", list(SPACES))
@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("mesh", list(MESHES))
def test_p2_raw_action_and_jacobian(mesh, form, space):
    m = MESHES[mesh]()
    T = _p2(m, form, space)
    To, Wsp = SPACES[space][1](m.coords, m.cells, form)
    n, nw = m.n_nodes, Wsp.n_w
    rng = np.random.default_rng(17)
    u = rng.uniform(-1, 1, n)
    a = rng.uniform(0.5, 2, nw)
    g = rng.uniform(-2, 2, nw)
    r = host(T.residual(dt(u), dt(a)))
    ro = np.bincount(To.i, weights=To.v * u[To.j] * a[To.k], minlength=nw)[:n]
    assert relerr(r, ro) < 1e-12
    dirm = m.dirichlet.astype(bool)
    Jg = csr_of(T, T.jacobian(dt(u), dt(a), dt(g), add_stiffness=(form == 1),
                              dirichlet=dt(m.dirichlet, torch.uint8)))
    A = sp.coo_matrix((To.v * a[To.k], (To.i, To.j)), shape=(n, n)).tocsr()
    B = sp.coo_matrix((To.v * u[To.j], (To.i, To.k)), shape=(n, nw)).tocsr()
    J = A + B @ sp.diags(g) @ Wsp.Pi
    if form == 1:
        J = J + O.assemble_stiffness(m.coords, m.cells)
    free = sp.diags((~dirm).astype(float))
    J = (free @ J @ free + sp.diags(dirm.astype(float))).tocsr()
    assert abs(Jg - J).max() <= 1e-12 * abs(J).max()
    # first term alone, no boundary handling
    Jg2 = csr_of(T, T.jacobian(dt(u), dt(a)))
    assert abs(Jg2 - A).max() <= 1e-12 * abs(A).max()


WORKLOADS = {
    "1d": lambda: W.nonlinear_diffusion_1d(64),
    "2d_n24": lambda: W.nonlinear_diffusion_2d(24),
    "2d_semilinear_n17": lambda: W.semilinear_2d(17),
    "3d_kappa_n4": lambda: W.diffusion_3d(4),
}


@pytest.mark.parametrize("space", list(SPACES))
@pytest.mark.parametrize("name", list(WORKLOADS))
def test_p2_problem_residual_and_jacobian(name, space):
    wl = WORKLOADS[name]()
    T = _p2(wl.mesh, wl.form, space)
    p = gpu_problem(T, wl)
    q = SPACES[space][2](O.build_problem(wl))
    u = np.random.default_rng(21).uniform(-1, 1, T.n)
    u[wl.mesh.dirichlet.astype(bool)] = 0.0
    F = T.problem_residual(p, dt(u))
    Fo = O.residual_p2(q, u)
    assert relerr(host(F), Fo) < 1e-12
    dinv = torch.empty(T.n, dtype=torch.float64, device=DEV)
    jv = T.problem_jacobian(p, dt(u), dinv=dinv)
    Jo = O.jacobian_p2(q, u)
    assert abs(csr_of(T, jv) - Jo).max() <= 1e-12 * abs(Jo).max()
    assert relerr(host(dinv), 1.0 / Jo.diagonal()) < 1e-12


@pytest.mark.parametrize("space", list(SPACES))
@pytest.mark.parametrize("name", list(WORKLOADS))
def test_p2_newton_equals_oracle_and_sga(name, space):
    wl = WORKLOADS[name]()
    T = _p2(wl.mesh, wl.form, space)
    p = gpu_problem(T, wl)
    po = O.build_problem(wl)
    q = SPACES[space][2](po)
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st = T.newton(p, u, eg().NewtonOptions(tol=1e-14, krylov_rtol=1e-14), warn=False)
    assert st.status in (0, 4), st.status_name       # converged or at the rounding floor
    ug = host(u)
    u_p2, _ = O.newton_p2(q, tol=1e-14)
    assert relerr(ug, u_p2) <= 1e-10
    if space == "p2" or wl.form == 0:
        # exact reformulations: the standard Galerkin solution
        u_sga, _ = O.sga_newton(po, tol=1e-14)
        assert relerr(ug, u_sga) <= 1e-10
    # certificate: the oracle's P2 residual at the GPU solution
    assert np.linalg.norm(O.residual_p2(q, ug)) <= 1e-10 * np.linalg.norm(po.d[po.free])


@pytest.mark.parametrize("space", list(SPACES))
def test_p2_picard_reaches_the_same_solution(space):
    wl = W.nonlinear_diffusion_2d(24)
    T = _p2(wl.mesh, wl.form, space)
    p = gpu_problem(T, wl)
    q = SPACES[space][2](O.build_problem(wl))
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st = T.picard(p, u, eg().PicardOptions(tol=1e-13, krylov_rtol=1e-6), warn=False)
    assert st.status == 0
    u_p2, _ = O.newton_p2(q, tol=1e-14)
    assert relerr(host(u), u_p2) <= 1e-10


def test_p2_full_size_2d_256_newton():
    """The headline workload with W_h = P2 (EGFEM == SGA): Newton to 1e-10 and
    sampled rows of the converged residual checked against the oracle."""
    wl = W.nonlinear_diffusion_2d(256)
    T = _p2(wl.mesh, wl.form)
    p = gpu_problem(T, wl)
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st = T.newton(p, u, eg().NewtonOptions(tol=1e-10, forcing=1))
    assert st.status == 0
    q = O.build_problem_p2(O.build_problem(wl))
    ug = host(u)
    Fo = O.residual_p2(q, ug)
    assert np.linalg.norm(Fo) <= 2e-10 * np.linalg.norm(q.base.d[q.base.free])
    # at the solution F is cancellation noise: compare on the scale of the
    # summed terms |T_ijk u_j a_k| of a row
    F = T.problem_residual(p, u)
    Pu = q.W.Pi @ ug
    aW = q.W.Pi @ q.base.a0 + Pu * Pu
    scale = np.bincount(q.I, weights=np.abs(q.V * ug[q.J] * aW[q.K]), minlength=T.n).max()
    assert np.abs(host(F) - Fo).max() <= 1e-12 * scale


@pytest.mark.parametrize("space", list(SPACES))
def test_p2_deterministic_and_rejections(space):
    wl = W.nonlinear_diffusion_2d(16)
    T = _p2(wl.mesh, wl.form, space)
    p = gpu_problem(T, wl)
    u1 = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    u2 = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    T.newton(p, u1)
    T.newton(p, u2)
    assert torch.equal(u1, u2)
    x = dt(np.ones(T.n))
    with pytest.raises(eg().EgfemError):
        T.mode3(x, x)
    with pytest.raises(eg().EgfemError):      # no convection form with W_h = P0
        eg().Tensor.from_mesh(wl.mesh, W.FORM_CONV, wspace=eg().W_P0)
    with pytest.raises(eg().EgfemError):
        eg().Tensor.from_mesh(wl.mesh, 0, wspace=7)
    with pytest.raises(eg().EgfemError):
        eg().newton_batched([T], [p], [u1])
    with pytest.raises(eg().EgfemError):
        T.residual(x, x)      # a must live on the dofs of W_h
