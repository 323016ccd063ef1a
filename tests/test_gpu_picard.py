"""Picard iteration (Sec. 4, Example picard_iteration) on the GPU against the
oracle: the SPD Picard matrix solved by Jacobi conjugate gradients (both
kernels) and the full iteration to its fixed point, which is also the Newton
solution."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import workloads as W
from oracle import egfem_oracle as O
from test_gpu_parity import DEV, csr_of, dt, eg, gpu_problem, host, relerr

pytestmark = pytest.mark.gpu

SMALL = {
    "1d": lambda: W.nonlinear_diffusion_1d(256),
    "2d_n40": lambda: W.nonlinear_diffusion_2d(40),
    "2d_semilinear_n33": lambda: W.semilinear_2d(33),
    "3d_kappa_n6": lambda: W.diffusion_3d(6),
}


@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("name", ["2d_n40", "3d_kappa_n6"])
def test_cg_solve_on_picard_matrix(name, kernel):
    """The Picard matrix A(u) emitted by egfem_jacobian (no a' term) equals the
    oracle's, and CG on it matches a direct solve."""
    wl = SMALL[name]()
    T = eg().Tensor.from_mesh(wl.mesh, wl.form)
    T.set_shape(krylov_kernel=kernel)
    po = O.build_problem(wl)
    u = np.random.default_rng(12).uniform(-1, 1, T.n)
    u[po.dirichlet] = 0.0
    a = po.a0 + u * u
    jv = T.jacobian(dt(u), dt(a), None, wl.add_stiffness, dt(wl.mesh.dirichlet, torch.uint8))
    Ao = O.picard_matrix(po, u)
    assert abs(csr_of(T, jv) - Ao).max() <= 1e-12 * abs(Ao).max()
    rhs = np.random.default_rng(13).uniform(-1, 1, T.n)
    x, rc, its, rr = T.solve_cg(jv, dt(rhs), rtol=1e-13)
    assert rc == 0, (rc, its, rr)
    xo = spla.spsolve(Ao.tocsc(), rhs)
    assert relerr(host(x), xo) < 1e-10
    assert relerr(Ao @ host(x), rhs) < 1e-12


def test_cg_reports_non_spd_breakdown():
    """A negative definite matrix makes the first curvature negative: status
    breakdown, no fault."""
    wl = W.nonlinear_diffusion_2d(12)
    T = eg().Tensor.from_mesh(wl.mesh, wl.form)
    n = T.n
    jv = T.jacobian(dt(np.zeros(n)), dt(np.ones(n)))
    x, rc, its, rr = T.solve_cg(-jv, dt(np.ones(n)), rtol=1e-12)
    assert rc == 2


@pytest.mark.parametrize("name", list(SMALL))
def test_picard_matches_oracle(name):
    wl = SMALL[name]()
    T = eg().Tensor.from_mesh(wl.mesh, wl.form)
    p = gpu_problem(T, wl)
    po = O.build_problem(wl)
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st = T.picard(p, u, eg().PicardOptions(tol=1e-13, krylov_rtol=1e-6), warn=False)
    assert st.status == 0, st.status_name
    up, sto = O.picard(po, tol=1e-13)
    un, _ = O.newton(po, tol=1e-14, max_iter=40)
    ug = host(u)
    assert relerr(ug, up) <= 1e-10
    assert relerr(ug, un) <= 1e-10
    assert np.linalg.norm(O.residual(po, ug)) <= 1e-10 * np.linalg.norm(po.d[po.free])
    # the contraction is the oracle's (inexact solves add at most a few steps)
    assert st.picard_iters <= sto.iterations + 5
    assert st.res <= 1e-10 * st.res0


@pytest.mark.parametrize("kernel,precond", [(0, 8), (0, 0), (1, 8), (2, 8)])
def test_picard_krylov_kernels(kernel, precond):
    """Resident CG with the block-Jacobi preconditioner (overlapped form,
    kernel 0, or barrier form, kernel 2) or the Jacobi preconditioner, and the
    streaming CG (Jacobi): the same Picard fixed point; the statistics name
    the kernel (bit 3: overlapped form)."""
    wl = W.nonlinear_diffusion_2d(40, seed=55)
    T = eg().Tensor.from_mesh(wl.mesh, wl.form)
    T.set_shape(krylov_kernel=kernel, krylov_precond=precond)
    p = gpu_problem(T, wl)
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st = T.picard(p, u, eg().PicardOptions(tol=1e-13), warn=False)
    assert st.status == 0
    assert st.krylov_kernels == {(0, 8): 13, (0, 0): 1, (1, 8): 2, (2, 8): 5}[(kernel, precond)]
    un, _ = O.newton(O.build_problem(wl), tol=1e-14)
    assert relerr(host(u), un) <= 1e-10


def test_picard_full_size_2d_256():
    """The 2D nonlinear-diffusion workload (66,049 nodes) to the paper's
    update tolerance."""
    wl = W.nonlinear_diffusion_2d(256)
    T = eg().Tensor.from_mesh(wl.mesh, wl.form)
    p = gpu_problem(T, wl)
    po = O.build_problem(wl)
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st = T.picard(p, u, eg().PicardOptions(tol=1e-12), warn=False)
    assert st.status == 0, st.status_name
    un, _ = O.newton(po, tol=1e-14, max_iter=30)
    ug = host(u)
    assert relerr(ug, un) <= 1e-10
    assert np.linalg.norm(O.residual(po, ug)) <= 1e-10 * np.linalg.norm(po.d[po.free])
    assert all(b < a for a, b in zip(st.update_hist[1:], st.update_hist[2:]))   # contracting


def test_picard_edge_cases():
    E = eg()
    wl = W.nonlinear_diffusion_2d(10)
    T = E.Tensor.from_mesh(wl.mesh, wl.form)
    dirm = dt(wl.mesh.dirichlet, torch.uint8)
    # zero load: the fixed point is u = 0, reached by the first solve
    p0 = E.Problem(T.n, torch.zeros(T.n, dtype=torch.float64, device=DEV), dirm, None, 1.0, False)
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st = T.picard(p0, u, warn=False)
    assert st.status == 0 and st.picard_iters == 1 and float(u.abs().max()) == 0.0
    # a non-finite guess is reported, not propagated as a fault
    p = gpu_problem(T, wl)
    u = torch.full((T.n,), float("nan"), dtype=torch.float64, device=DEV)
    st = T.picard(p, u, warn=False)
    assert st.status == 3
    # a step whose solve turns non-finite (load 1e120: the first iterate is
    # ~1e120, so the next matrix times it overflows) ends the iteration with u
    # at the last finite iterate
    big = E.Problem(T.n, p.load * 1e120, dirm, None, 1.0, False)
    u1 = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st1 = T.picard(big, u1, E.PicardOptions(max_picard=1), warn=False)
    assert st1.status == 1 and bool(torch.isfinite(u1).all()) and float(u1.abs().max()) > 1e100
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st = T.picard(big, u, warn=False)
    assert st.status == 3 and st.picard_iters == 2, (st.status_name, st.picard_iters)
    assert torch.equal(u, u1)
    # iteration cap
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st = T.picard(p, u, E.PicardOptions(max_picard=2), warn=False)
    assert st.status == 1 and st.picard_iters == 2
    # warm start from the fixed point: one step, negligible update
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    T.picard(p, u, E.PicardOptions(tol=1e-13), warn=False)
    st = T.picard(p, u, E.PicardOptions(tol=1e-11), warn=False)
    assert st.status == 0 and st.picard_iters == 1


@pytest.mark.parametrize("kernel,precond", [(0, 8), (1, 0)])
def test_picard_timing_leaves_the_iteration_unchanged(kernel, precond):
    """Each Picard step reads the CG outcome, its timing events and the update
    norms in one synchronisation: with timing on, the iterate is bitwise the
    untimed one, the per-step CG counts add up to the total and the CG time is
    reported."""
    wl = W.nonlinear_diffusion_2d(40, seed=56)
    T = eg().Tensor.from_mesh(wl.mesh, wl.form)
    T.set_shape(krylov_kernel=kernel, krylov_precond=precond)
    p = gpu_problem(T, wl)
    runs = []
    for timing in (0, 1, 0):
        u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
        st = T.picard(p, u, eg().PicardOptions(tol=1e-13, timing=timing), warn=False)
        assert st.status == 0, st.status_name
        assert st.picard_iters <= 64 and sum(st.krylov_hist) == st.krylov_iters
        assert (st.t_krylov_ms > 0.0) == bool(timing)
        runs.append((u, st))
    (u0, s0), (u1, s1), (u2, s2) = runs
    assert torch.equal(u0, u1) and torch.equal(u0, u2)
    assert s0.picard_iters == s1.picard_iters == s2.picard_iters
    assert s0.krylov_hist == s1.krylov_hist == s2.krylov_hist
    assert s0.update_hist == s1.update_hist
    un, _ = O.newton(O.build_problem(wl), tol=1e-14)
    assert relerr(host(u1), un) <= 1e-10
