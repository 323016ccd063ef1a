"""High-valence unstructured mesh: a wheel whose centre node has k neighbours
(free inner ring, Dirichlet outer ring).  Rows longer than 16 entries take the
streaming Krylov row shapes with several lanes per row, and k = 150 exceeds
what two entries per lane cover (the tail loop).  Newton, BiCGStab, CG /
Picard and the batched kernel against the oracle."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import workloads as W
from oracle import egfem_oracle as O
from test_gpu_parity import DEV, csr_of, dt, eg, host, relerr

pytestmark = pytest.mark.gpu


def wheel(k, seed=9):
    rng = np.random.default_rng(seed)
    t = 2 * np.pi * (np.arange(k) + rng.uniform(-0.2, 0.2, k)) / k
    inner = np.stack([0.5 * np.cos(t), 0.5 * np.sin(t)], 1)
    outer = np.stack([np.cos(t + np.pi / k), np.sin(t + np.pi / k)], 1)
    coords = np.vstack([[[0.0, 0.0]], inner, outer])
    cells = []
    for i in range(k):
        a, b = 1 + i, 1 + (i + 1) % k
        A, B = 1 + k + i, 1 + k + (i + 1) % k
        cells += [[0, a, b], [a, A, b], [b, A, B]]
    dirm = np.zeros(2 * k + 1, dtype=np.uint8)
    dirm[1 + k:] = 1
    mesh = W.Mesh(2, k, coords, np.array(cells, dtype=np.int32), dirm)
    f = rng.uniform(0, 10, 2 * k + 1)
    return W.Workload(f"wheel_{k}", mesh, f, O.FORM_STIFF, None, 1.0, False, 1e-12, seed)


def device(T, wl):
    load = T.matvec(dt(wl.f), "M")
    return eg().Problem(T.n, load, dt(wl.mesh.dirichlet, torch.uint8), None, 1.0, False)


@pytest.mark.parametrize("k", [40, 150])
def test_wheel_newton_solve_picard(k):
    wl = wheel(k)
    T = eg().Tensor.build(wl.mesh.coords, wl.mesh.cells, wl.form)
    assert T.info.n_nodes == 2 * k + 1
    p = device(T, wl)
    po = O.build_problem(wl)
    un, _ = O.newton(po, tol=1e-14)
    for kernel in (0, 1):
        T.set_shape(krylov_kernel=kernel)
        u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
        st = T.newton(p, u, eg().NewtonOptions(tol=1e-14, krylov_rtol=1e-14, max_newton=40), warn=False)
        assert st.status in (0, 4), st.status_name
        assert st.krylov_kernels == 2           # rows of k + 1 entries: always the streaming kernel
        assert relerr(host(u), un) <= 1e-10
        u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
        sp_ = T.picard(p, u, eg().PicardOptions(tol=1e-13), warn=False)
        assert sp_.status == 0 and relerr(host(u), un) <= 1e-10
    # BiCGStab on DF and CG on the Picard matrix against SuperLU
    ur = np.random.default_rng(2).uniform(-1, 1, T.n)
    ur[po.dirichlet] = 0.0
    rhs = np.random.default_rng(3).uniform(-1, 1, T.n)
    jv = T.problem_jacobian(p, dt(ur))
    x, rc, its, rr = T.solve(jv, dt(rhs), rtol=1e-13)
    assert rc == 0 and relerr(host(x), spla.spsolve(O.jacobian(po, ur).tocsc(), rhs)) < 1e-9
    A = O.picard_matrix(po, ur)
    ja = T.jacobian(dt(ur), dt(po.a0 + ur * ur), None, False, dt(wl.mesh.dirichlet, torch.uint8))
    assert abs(csr_of(T, ja) - A).max() <= 1e-12 * abs(A).max()
    x, rc, its, rr = T.solve_cg(ja, dt(rhs), rtol=1e-13)
    assert rc == 0 and relerr(host(x), spla.spsolve(A.tocsc(), rhs)) < 1e-10


def test_wheel_batched_with_grid_instances():
    """The launch's row shape follows the longest row of any instance."""
    E = eg()
    wls = [wheel(40), wheel(150, seed=4), W.nonlinear_diffusion_2d(20)]
    Ts = [E.Tensor.build(w.mesh.coords, w.mesh.cells, w.form) for w in wls]
    Ps = [device(T, w) for T, w in zip(Ts, wls)]
    us = [torch.zeros(T.n, dtype=torch.float64, device=DEV) for T in Ts]
    opts = E.NewtonOptions(tol=1e-14, krylov_rtol=1e-14, max_newton=40)
    stats, rc = E.newton_batched(Ts, Ps, us, opts)
    assert rc in (0, 4)
    for w, u, s in zip(wls, us, stats):
        assert s.status in (0, 4), (w.name, s.status_name)
        un, _ = O.newton(O.build_problem(w), tol=1e-14)
        assert relerr(host(u), un) <= 1e-10, w.name


def test_wheel_neighbour_list_overflow_takes_team_barrier():
    """64 workgroups on a wheel with 150 rim nodes (some workgroups get no rows):
    the hub's workgroup gathers from 33 others, more than a neighbour list
    holds, so every workgroup
    synchronises through the team barrier (a mix of the two kinds of wait would
    never complete).  BiCGStab and CG against SuperLU, deterministic."""
    wl = wheel(150, seed=5)
    T = eg().Tensor.build(wl.mesh.coords, wl.mesh.cells, wl.form)
    p = device(T, wl)
    po = O.build_problem(wl)
    ur = np.random.default_rng(6).uniform(-1, 1, T.n)
    ur[po.dirichlet] = 0.0
    rhs = np.random.default_rng(7).uniform(-1, 1, T.n)
    jv = T.problem_jacobian(p, dt(ur))
    A = O.picard_matrix(po, ur)
    ja = T.jacobian(dt(ur), dt(po.a0 + ur * ur), None, False, dt(wl.mesh.dirichlet, torch.uint8))
    for threads in (256, 1024):
        print(f"wheel 150 overflow grid=64x{threads}", flush=True)
        T.set_shape(krylov_blocks=64, krylov_threads=threads)
        x, rc, its, rr = T.solve(jv, dt(rhs), rtol=1e-13)
        assert rc == 0 and relerr(host(x), spla.spsolve(O.jacobian(po, ur).tocsc(), rhs)) < 1e-9
        x2, _, its2, _ = T.solve(jv, dt(rhs), rtol=1e-13)
        assert its2 == its and torch.equal(x, x2)
        x, rc, its, rr = T.solve_cg(ja, dt(rhs), rtol=1e-13)
        assert rc == 0 and relerr(host(x), spla.spsolve(A.tocsc(), rhs)) < 1e-10
