"""Viscous Burgers' equation (Sec. 5.2) on the GPU against the oracle: the
convection tensor N, the constant system matrix M + dt nu K, and the
semi-implicit steps in the tensor (N:(u (x) u)) and group (N^f (u . u))
formulations, at the paper's settings (nu = 1, T = 1, dt = 1e-2)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import egfem_oracle as O
from test_gpu_parity import DEV, dt, eg, host, irregular_mesh, relerr

pytestmark = pytest.mark.gpu


def _oracle(mesh, u0, source, dt_, nu, steps, group):
    sy = O.burgers_system(mesh.coords, mesh.cells, mesh.dirichlet, dt_, nu)
    return O.burgers(sy, u0, source, steps, group=group)


def _smooth_case(mesh, seed):
    """Seeded initial value (zero on the boundary) and one constant source."""
    rng = np.random.default_rng(seed)
    u0 = rng.uniform(-1.0, 1.0, mesh.n_nodes) * (mesh.dirichlet == 0)
    src = rng.uniform(-5.0, 5.0, mesh.n_nodes)
    return u0, src


@pytest.mark.parametrize("group", [0, 1])
@pytest.mark.parametrize("n", [16, 40])
def test_burgers_manufactured_matches_oracle(n, group):
    print(f"burgers manufactured n={n} group={group}", flush=True)
    b = W.burgers_2d(n)
    T = eg().Tensor.from_mesh(b.mesh, W.FORM_CONV)
    u = dt(b.u0)
    st = T.burgers(u, dt(b.mesh.dirichlet, torch.uint8), dt(b.source),
                   eg().BurgersOptions(dt=b.dt, nu=b.nu, steps=b.steps, group=group, krylov_rtol=1e-13))
    assert st.status == 0, st.status_name
    assert st.steps == b.steps and st.krylov_iters > 0 and st.max_relres <= 1e-13
    uo = _oracle(b.mesh, b.u0, b.source, b.dt, b.nu, b.steps, bool(group))
    ug = host(u)
    assert relerr(ug, uo) < 1e-11
    # both are the same discretisation of the manufactured solution
    err = np.linalg.norm(ug - b.u_final) / np.linalg.norm(b.u_final)
    assert err < (1e-2 if n == 16 else 2e-3)


MESHES = {
    "1d_n64": (lambda: W.mesh_1d(64), 30),
    "2d_jitter_n21": (lambda: irregular_mesh(21), 30),
    "3d_n5": (lambda: W.mesh_3d(5), 10),
}


@pytest.mark.parametrize("group", [0, 1])
@pytest.mark.parametrize("name", list(MESHES))
def test_burgers_other_meshes(name, group):
    print(f"burgers mesh={name} group={group}", flush=True)
    mk, steps = MESHES[name]
    m = mk()
    T = eg().Tensor.from_mesh(m, W.FORM_CONV)
    u0, src = _smooth_case(m, 31)
    u = dt(u0)
    st = T.burgers(u, dt(m.dirichlet, torch.uint8), dt(src),
                   eg().BurgersOptions(dt=0.02, nu=0.3, steps=steps, group=group, krylov_rtol=1e-13))
    assert st.status == 0, st.status_name
    uo = _oracle(m, u0, np.broadcast_to(src, (steps, m.n_nodes)), 0.02, 0.3, steps, bool(group))
    assert relerr(host(u), uo) < 1e-11


@pytest.mark.parametrize("kernel,precond", [(0, 8), (0, 0), (1, 8), (2, 8)])
def test_burgers_krylov_kernels_and_determinism(kernel, precond):
    b = W.burgers_2d(32, dt=2e-2)
    T = eg().Tensor.from_mesh(b.mesh, W.FORM_CONV)
    T.set_shape(krylov_kernel=kernel, krylov_precond=precond)
    dirm = dt(b.mesh.dirichlet, torch.uint8)
    src = dt(b.source)
    o = eg().BurgersOptions(dt=b.dt, steps=b.steps, krylov_rtol=1e-13, timing=1)
    u1 = dt(b.u0)
    s1 = T.burgers(u1, dirm, src, o)
    u2 = dt(b.u0)
    s2 = T.burgers(u2, dirm, src, o)
    assert s1.status == 0 and s1.krylov_kernels == {(0, 8): 13, (0, 0): 1, (1, 8): 2, (2, 8): 5}[(kernel, precond)]
    assert torch.equal(u1, u2) and s1.krylov_hist == s2.krylov_hist
    assert s1.t_krylov_ms > 0.0 and s1.t_rhs_ms > 0.0
    uo = _oracle(b.mesh, b.u0, b.source, b.dt, b.nu, b.steps, False)
    assert relerr(host(u1), uo) < 1e-11


def test_burgers_full_size_2d_256():
    """The benchmark configuration: 2D 256x256, 100 steps, default options."""
    print("burgers 2d_256 full size", flush=True)
    b = W.burgers_2d(256)
    T = eg().Tensor.from_mesh(b.mesh, W.FORM_CONV)
    dirm = dt(b.mesh.dirichlet, torch.uint8)
    src = dt(b.source)
    for group in (0, 1):
        u = dt(b.u0)
        st = T.burgers(u, dirm, src, eg().BurgersOptions(group=group))
        assert st.status == 0 and st.steps == 100
        uo = _oracle(b.mesh, b.u0, b.source, b.dt, b.nu, b.steps, bool(group))
        assert relerr(host(u), uo) < 1e-9
        assert np.linalg.norm(host(u) - b.u_final) / np.linalg.norm(b.u_final) < 1e-3


def test_burgers_edge_cases():
    m = W.mesh_2d(12)
    T = eg().Tensor.from_mesh(m, W.FORM_CONV)
    dirm = dt(m.dirichlet, torch.uint8)
    u0, src = _smooth_case(m, 5)
    # zero steps: only the Dirichlet entries are zeroed
    raw = u0 + 3.0 * m.dirichlet
    u = dt(raw)
    st = T.burgers(u, dirm, None, eg().BurgersOptions(steps=0))
    assert st.status == 0 and st.steps == 0
    assert np.array_equal(host(u), u0)
    # zero initial value and no source stay zero, without CG iterations
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st = T.burgers(u, dirm, None, eg().BurgersOptions(steps=5))
    assert st.status == 0 and st.krylov_iters == 0 and not torch.any(u)
    # a [steps, n] source with equal rows equals the same vector with stride 0
    o = eg().BurgersOptions(steps=4, krylov_rtol=1e-13)
    ua, ub = dt(u0), dt(u0)
    T.burgers(ua, dirm, dt(src), o)
    T.burgers(ub, dirm, dt(np.tile(src, (4, 1))), o)
    assert torch.equal(ua, ub)
    # no Dirichlet nodes at all (natural boundary): still SPD (mass term)
    uc = dt(u0)
    st = T.burgers(uc, None, dt(src), o)
    assert st.status == 0
    sy = O.burgers_system(m.coords, m.cells, np.zeros(m.n_nodes, np.uint8), o.dt, o.nu)
    assert relerr(host(uc), O.burgers(sy, u0, np.tile(src, (4, 1)), 4)) < 1e-11
    # non-finite initial value: status non-finite after the first step
    bad = u0.copy()
    bad[m.n_nodes // 2] = np.nan
    st = T.burgers(dt(bad), dirm, None, eg().BurgersOptions(steps=5), warn=False)
    assert st.status == 3 and st.steps == 1
    # wrong tensor form and bad options are argument errors
    S = eg().Tensor.from_mesh(m, W.FORM_STIFF)
    with pytest.raises(eg().EgfemError):
        S.burgers(dt(u0), dirm)
    with pytest.raises(eg().EgfemError):
        T.burgers(dt(u0), dirm, None, eg().BurgersOptions(dt=0.0))
    with pytest.raises(eg().EgfemError):
        T.burgers(dt(u0), dirm, dt(np.tile(src, (2, 1))), eg().BurgersOptions(steps=3))


def test_burgers_initial_guess_orders():
    """Extrapolated initial iterates change the CG work, not the answer."""
    b = W.burgers_2d(32)
    T = eg().Tensor.from_mesh(b.mesh, W.FORM_CONV)
    dirm = dt(b.mesh.dirichlet, torch.uint8)
    src = dt(b.source)
    uo = _oracle(b.mesh, b.u0, b.source, b.dt, b.nu, 30, False)
    iters = []
    for guess in (0, 1, 2):
        u = dt(b.u0)
        st = T.burgers(u, dirm, src, eg().BurgersOptions(steps=30, guess=guess, krylov_rtol=1e-13))
        assert st.status == 0
        assert relerr(host(u), uo) < 1e-11
        iters.append(st.krylov_iters)
    assert iters[2] < iters[1] < iters[0], iters
    with pytest.raises(eg().EgfemError):
        T.burgers(dt(b.u0), dirm, src, eg().BurgersOptions(steps=3, guess=3))


P2_MESHES = {
    "1d_n16": lambda: W.mesh_1d(16),
    "2d_n9": lambda: W.mesh_2d(9),
    "2d_jitter_n13": lambda: irregular_mesh(13),
    "3d_n3": lambda: W.mesh_3d(3),
}


@pytest.mark.parametrize("name", list(P2_MESHES))
def test_burgers_p2_convection_tensor_matches_oracle(name):
    """The W_h = P2 convection tensor entry by entry."""
    m = P2_MESHES[name]()
    print(f"burgers p2 tensor mesh={name}", flush=True)
    T = eg().Tensor.from_mesh(m, W.FORM_CONV, wspace=eg().W_P2)
    To, Wsp = O.tensor_p2(m.coords, m.cells, O.FORM_CONV)
    assert T.info.wspace == eg().W_P2 and T.info.n_w == Wsp.n_w
    assert T.info.nnz == To.nnz and T.info.structural_nnz == To.structural_nnz
    i, j, k, v = T.export()
    nw = Wsp.n_w
    kg = (i.astype(np.int64) * nw + j) * nw + k
    ko = (To.i * nw + To.j) * nw + To.k
    og, oo = np.argsort(kg), np.argsort(ko)
    assert np.array_equal(kg[og], ko[oo])
    assert np.abs(v[og] - To.v[oo]).max() <= 1e-14 * np.abs(To.v).max()


@pytest.mark.parametrize("name", ["1d_n16", "2d_jitter_n13", "3d_n3"])
def test_burgers_p2_group_matches_oracle(name):
    """EGFEM group formulation with W_h = P2: N^f_P2 (Pi u)^2 on the GPU against
    the oracle's, and against the tensor formulation N:(u (x) u), which it
    reproduces exactly (u^2 of a P1 u lies in P2)."""
    m = P2_MESHES[name]()
    print(f"burgers p2 group mesh={name}", flush=True)
    steps = 12
    T = eg().Tensor.from_mesh(m, W.FORM_CONV, wspace=eg().W_P2)
    u0, src = _smooth_case(m, 44)
    u = dt(u0)
    o = eg().BurgersOptions(dt=0.02, nu=0.3, steps=steps, group=1, krylov_rtol=1e-13)
    st = T.burgers(u, dt(m.dirichlet, torch.uint8), dt(src), o)
    assert st.status == 0 and st.steps == steps
    sy = O.burgers_system(m.coords, m.cells, m.dirichlet, 0.02, 0.3)
    srcs = np.broadcast_to(src, (steps, m.n_nodes))
    uo = O.burgers(sy, u0, srcs, steps, group_p2=O.burgers_group_p2(m.coords, m.cells))
    assert relerr(host(u), uo) < 1e-11
    ut = O.burgers(sy, u0, srcs, steps, group=False)
    assert relerr(host(u), ut) < 1e-11


def test_burgers_p2_full_size_2d_256_and_rejections():
    """The 2D 256x256 manufactured run with W_h = P2 equals the tensor
    formulation; a P2 convection tensor rejects the slot (P1) group form."""
    print("burgers p2 2d_256 full size", flush=True)
    b = W.burgers_2d(256)
    dirm = dt(b.mesh.dirichlet, torch.uint8)
    src = dt(b.source)
    T = eg().Tensor.from_mesh(b.mesh, W.FORM_CONV, wspace=eg().W_P2)
    u = dt(b.u0)
    st = T.burgers(u, dirm, src, eg().BurgersOptions(group=1))
    assert st.status == 0 and st.steps == 100
    uo = _oracle(b.mesh, b.u0, b.source, b.dt, b.nu, b.steps, False)
    assert relerr(host(u), uo) < 1e-9
    assert np.linalg.norm(host(u) - b.u_final) / np.linalg.norm(b.u_final) < 1e-3
    with pytest.raises(eg().EgfemError):
        T.burgers(dt(b.u0), dirm, src, eg().BurgersOptions(group=0))
    # the P0 space has no convection tensor
    with pytest.raises(eg().EgfemError):
        eg().Tensor.from_mesh(W.mesh_2d(6), W.FORM_CONV, wspace=eg().W_P0)


@pytest.mark.parametrize("name", list(P2_MESHES))
def test_burgers_iq_convection_tensor_matches_oracle(name):
    """The W_h = I_k convection tensor (w_q |e| phi_j(x_q) sum_d d_d phi_i)
    entry by entry."""
    m = P2_MESHES[name]()
    print(f"burgers iq tensor mesh={name}", flush=True)
    T = eg().Tensor.from_mesh(m, W.FORM_CONV, wspace=eg().W_IQ)
    To, Wsp = O.tensor_iq(m.coords, m.cells, O.FORM_CONV)
    assert T.info.wspace == eg().W_IQ and T.info.n_w == Wsp.n_w
    assert T.info.nnz == To.nnz and T.info.structural_nnz == To.structural_nnz
    i, j, k, v = T.export()
    nw = Wsp.n_w
    kg = (i.astype(np.int64) * nw + j) * nw + k
    ko = (To.i * nw + To.j) * nw + To.k
    og, oo = np.argsort(kg), np.argsort(ko)
    assert np.array_equal(kg[og], ko[oo])
    assert np.abs(v[og] - To.v[oo]).max() <= 1e-14 * np.abs(To.v).max()


@pytest.mark.parametrize("name", ["1d_n16", "2d_jitter_n13", "3d_n3"])
def test_burgers_iq_group_matches_oracle(name):
    """EGFEM group formulation with W_h = I_k: N^f_I (Pi u)^2, u_h squared at
    the points, on the GPU against the oracle's, and against the tensor
    formulation, which it reproduces (the rules integrate u_h^2 exactly)."""
    m = P2_MESHES[name]()
    print(f"burgers iq group mesh={name}", flush=True)
    steps = 12
    T = eg().Tensor.from_mesh(m, W.FORM_CONV, wspace=eg().W_IQ)
    u0, src = _smooth_case(m, 45)
    u = dt(u0)
    o = eg().BurgersOptions(dt=0.02, nu=0.3, steps=steps, group=1, krylov_rtol=1e-13)
    st = T.burgers(u, dt(m.dirichlet, torch.uint8), dt(src), o)
    assert st.status == 0 and st.steps == steps
    sy = O.burgers_system(m.coords, m.cells, m.dirichlet, 0.02, 0.3)
    srcs = np.broadcast_to(src, (steps, m.n_nodes))
    uo = O.burgers(sy, u0, srcs, steps, group_p2=O.burgers_group_iq(m.coords, m.cells))
    assert relerr(host(u), uo) < 1e-11
    ut = O.burgers(sy, u0, srcs, steps, group=False)
    assert relerr(host(u), ut) < 1e-11


def test_burgers_iq_full_size_2d_256_and_rejections():
    """The 2D 256x256 manufactured run with W_h = I_3 (the 3-point rule)
    equals the tensor formulation; an I_k convection tensor rejects the slot
    (P1) group form and the tensor formulation."""
    print("burgers iq 2d_256 full size", flush=True)
    b = W.burgers_2d(256)
    dirm = dt(b.mesh.dirichlet, torch.uint8)
    src = dt(b.source)
    T = eg().Tensor.from_mesh(b.mesh, W.FORM_CONV, wspace=eg().W_IQ)
    assert T.info.n_w == 3 * b.mesh.cells.shape[0]
    u = dt(b.u0)
    st = T.burgers(u, dirm, src, eg().BurgersOptions(group=1))
    assert st.status == 0 and st.steps == 100
    uo = _oracle(b.mesh, b.u0, b.source, b.dt, b.nu, b.steps, False)
    assert relerr(host(u), uo) < 1e-9
    assert np.linalg.norm(host(u) - b.u_final) / np.linalg.norm(b.u_final) < 1e-3
    with pytest.raises(eg().EgfemError):
        T.burgers(dt(b.u0), dirm, src, eg().BurgersOptions(group=0))
