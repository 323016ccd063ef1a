"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances (FP64): per-call outputs (tensor entries, actions, Jacobian values,
matrix-vector products) differ only by summation order, so they are compared
normwise at 1e-12 relative (observed ~1e-15).  Converged Newton solutions are
compared at 1e-10 relative with both sides iterated to their rounding floor,
plus a certificate: the oracle's residual evaluated at the GPU solution.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import torch

import workloads as W
from oracle import egfem_oracle as O

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def eg():
    import paper_2005_06193_amd as mod
    return mod


def dt(x, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def gpu_problem(T, wl):
    """Device problem with the load d = M f computed on the GPU."""
    f = dt(wl.f)
    load = T.matvec(f, "M")
    dirm = dt(wl.mesh.dirichlet, torch.uint8)
    a0 = dt(wl.a0) if wl.a0 is not None else None
    return eg().Problem(T.n, load, dirm, a0, wl.a0_const, wl.add_stiffness)


def csr_of(T, jval):
    rp, cl = T.pattern()
    return sp.csr_matrix((host(jval), cl, rp), shape=(T.n, T.n))


def relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def irregular_mesh(n, seed=3):
    """Structured 2D mesh with jittered interior nodes (non-uniform elements)."""
    m = W.mesh_2d(n)
    rng = np.random.default_rng(seed)
    c = m.coords.copy()
    inner = m.dirichlet == 0
    c[inner] += rng.uniform(-0.25, 0.25, size=(inner.sum(), 2)) / n
    return W.Mesh(2, n, c, m.cells, m.dirichlet)


MESHES = {
    "1d_n16": lambda: W.mesh_1d(16),
    "1d_n257": lambda: W.mesh_1d(257),
    "2d_n8": lambda: W.mesh_2d(8),
    "2d_n37": lambda: W.mesh_2d(37),
    "2d_jitter_n21": lambda: irregular_mesh(21),
    "3d_n3": lambda: W.mesh_3d(3),
    "3d_n7": lambda: W.mesh_3d(7),
}


# ---------------------------------------------------------------------------
# offline build
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mesh", list(MESHES))
@pytest.mark.parametrize("form", [0, 1, 2])
def test_build_matches_oracle_tensor(mesh, form):
    m = MESHES[mesh]()
    T = eg().Tensor.from_mesh(m, form)
    To = O.assemble_tensor(m.coords, m.cells, form)
    i, j, k, v = T.export()
    assert T.info.nnz == To.nnz
    assert T.info.structural_nnz == To.structural_nnz
    key_g = (i.astype(np.int64) * m.n_nodes + j) * m.n_nodes + k
    key_o = (To.i * m.n_nodes + To.j) * m.n_nodes + To.k
    og = np.argsort(key_g)
    oo = np.argsort(key_o)
    assert np.array_equal(key_g[og], key_o[oo])
    assert np.abs(v[og] - To.v[oo]).max() <= 1e-14 * np.abs(To.v).max()
    # stiffness and mass matrices in the pattern
    x = np.random.default_rng(1).uniform(-1, 1, m.n_nodes)
    K = O.assemble_stiffness(m.coords, m.cells)
    M = O.assemble_mass(m.coords, m.cells)
    assert relerr(host(T.matvec(dt(x), "K")), K @ x) < 1e-13
    assert relerr(host(T.matvec(dt(x), "M")), M @ x) < 1e-13


def test_build_counts_full_size():
    """Stored / structural entries and slots at the full workload sizes."""
    for n in (256, 512):
        m = W.mesh_2d(n)
        T = eg().Tensor.from_mesh(m, 0)
        assert T.info.nnz == 23 * n * n + 14 * n + 1
        assert T.info.structural_nnz == 31 * n * n + 14 * n + 1
        assert T.info.slots == 7 * n * n + 6 * n + 1
        T.close()
    m = W.mesh_2d(512)
    T = eg().Tensor.from_mesh(m, 1)
    assert T.info.nnz == 31 * 512 ** 2 + 14 * 512 + 1
    T.close()
    n = 64
    m = W.mesh_3d(n)
    T = eg().Tensor.from_mesh(m, 0)
    assert T.info.nnz == 63 * n ** 3 + 69 * n ** 2 + 21 * n + 1
    assert T.info.structural_nnz == 115 * n ** 3 + 93 * n ** 2 + 21 * n + 1
    assert T.info.slots == 4018753
    T.close()


# ---------------------------------------------------------------------------
# tensor actions
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mesh", list(MESHES))
@pytest.mark.parametrize("form", [0, 1, 2])
def test_raw_action_and_mode3(mesh, form):
    m = MESHES[mesh]()
    T = eg().Tensor.from_mesh(m, form)
    To = O.assemble_tensor(m.coords, m.cells, form)
    rng = np.random.default_rng(7)
    u = rng.uniform(-1, 1, m.n_nodes)
    a = rng.uniform(0.5, 2, m.n_nodes)
    w = rng.uniform(-1, 1, m.n_nodes)
    r = host(T.residual(dt(u), dt(a)))
    assert relerr(r, O.contract_uv(To, u, a)) < 1e-12
    q = host(T.mode3(dt(w), dt(u)))
    assert relerr(q, O.contract_mode3(To, w, u)) < 1e-12


@pytest.mark.parametrize("mesh", list(MESHES))
@pytest.mark.parametrize("form", [0, 1, 2])
def test_jacobian_emission(mesh, form):
    m = MESHES[mesh]()
    T = eg().Tensor.from_mesh(m, form)
    To = O.assemble_tensor(m.coords, m.cells, form)
    rng = np.random.default_rng(8)
    u = rng.uniform(-1, 1, m.n_nodes)
    a = rng.uniform(0.5, 2, m.n_nodes)
    g = rng.uniform(-2, 2, m.n_nodes)
    dirm = m.dirichlet.astype(bool)
    Jg = csr_of(T, T.jacobian(dt(u), dt(a), dt(g), add_stiffness=(form == 1),
                              dirichlet=dt(m.dirichlet, torch.uint8)))
    J = O.contract_first(To, a) + O.contract_mode2(To, u) @ sp.diags(g)
    if form == 1:
        J = J + O.assemble_stiffness(m.coords, m.cells)
    free = sp.diags((~dirm).astype(float))
    J = (free @ J @ free + sp.diags(dirm.astype(float))).tocsr()
    assert abs(Jg - J).max() <= 1e-12 * abs(J).max()
    # without the second term and without boundary handling
    Jg2 = csr_of(T, T.jacobian(dt(u), dt(a)))
    assert abs(Jg2 - O.contract_first(To, a)).max() <= 1e-12 * abs(J).max()
    # transposed product through the slot permutation
    x = rng.uniform(-1, 1, m.n_nodes)
    jv = T.jacobian(dt(u), dt(a), dt(g))
    Jf = O.contract_first(To, a) + O.contract_mode2(To, u) @ sp.diags(g)
    assert relerr(host(T.matvec(dt(x), "J", jval=jv, transpose=True)), Jf.T @ x) < 1e-12
    assert relerr(host(T.matvec(dt(x), "J", jval=jv)), Jf @ x) < 1e-12


WORKLOADS_SMALL = {
    "1d": lambda: W.nonlinear_diffusion_1d(256),
    "2d_n40": lambda: W.nonlinear_diffusion_2d(40),
    "2d_semilinear_n33": lambda: W.semilinear_2d(33),
    "3d_kappa_n6": lambda: W.diffusion_3d(6),
}


@pytest.mark.parametrize("name", list(WORKLOADS_SMALL))
def test_problem_residual_and_jacobian(name):
    wl = WORKLOADS_SMALL[name]()
    T = eg().Tensor.from_mesh(wl.mesh, wl.form)
    p = gpu_problem(T, wl)
    po = O.build_problem(wl)
    assert relerr(host(p.load), po.d) < 1e-13
    u = np.random.default_rng(9).uniform(-1, 1, T.n)
    u[po.dirichlet] = 0
    F, nrm = T.problem_residual(p, dt(u), with_norm=True)
    Fo = O.residual(po, u)
    assert relerr(host(F), Fo) < 1e-12
    assert abs(nrm - np.linalg.norm(Fo)) <= 1e-12 * np.linalg.norm(Fo)
    dinv = torch.empty(T.n, dtype=torch.float64, device=DEV)
    Jg = csr_of(T, T.problem_jacobian(p, dt(u), dinv=dinv))
    Jo = O.jacobian(po, u)
    assert abs(Jg - Jo).max() <= 1e-12 * abs(Jo).max()
    assert relerr(host(dinv), 1.0 / Jo.diagonal()) < 1e-12


# ---------------------------------------------------------------------------
# linear solve
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kernel", [0, 1, 2])
@pytest.mark.parametrize("transpose", [False, True])
def test_bicgstab_solve(transpose, kernel):
    """The BiCGStab kernels: 0 = register-resident (every workgroup's rows
    fit its threads here; overlapped form with the block preconditioner),
    1 = streaming, 2 = register-resident in the barrier form."""
    wl = W.nonlinear_diffusion_2d(48)
    T = eg().Tensor.from_mesh(wl.mesh, wl.form)
    T.set_shape(krylov_kernel=kernel)
    p = gpu_problem(T, wl)
    po = O.build_problem(wl)
    u = np.random.default_rng(10).uniform(0, 1, T.n)
    u[po.dirichlet] = 0
    jv = T.problem_jacobian(p, dt(u))
    Jo = O.jacobian(po, u)
    rhs = np.random.default_rng(11).uniform(-1, 1, T.n)
    x, rc, its, rr = T.solve(jv, dt(rhs), transpose=transpose, rtol=1e-13)
    assert rc == 0, (rc, its, rr)
    A = (Jo.T if transpose else Jo).tocsc()
    xo = spla.spsolve(A, rhs)
    # ||x - x*|| <= cond * rtol; cond(J) ~ 1e3 here
    assert relerr(host(x), xo) < 1e-9
    assert relerr(A @ host(x), rhs) < 1e-12


BJ_MESHES = {
    "1d_n120": lambda: W.mesh_1d(120),
    "2d_jitter_n45": lambda: irregular_mesh(45),
    "disk_n40": lambda: W.mesh_disk(40),
    # rows of up to 15 entries: the 1024-thread resident form (8 entries in
    # registers, the rest in LDS) on every row; 256/512 threads stream
    "3d_n9": lambda: W.mesh_3d(9),
}


@pytest.mark.parametrize("kernel", [0, 2])
@pytest.mark.parametrize("precond", [0, 2, 8, 32])
@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("mesh", list(BJ_MESHES))
def test_bicgstab_block_preconditioner(mesh, transpose, precond, kernel):
    """BiCGStab with the block-Jacobi preconditioner (k Chebyshev steps on each
    workgroup's block of a coordinate-bisection partition) against SuperLU on
    a nonsymmetric Newton Jacobian, for several grids and workgroup sizes, in
    the overlapped form (kernel 0: flag-in-data synchronisation) and the
    barrier form (kernel 2); deterministic; fewer iterations than Jacobi.
    (The uniform fallback to the team barrier when a part has too many
    neighbours runs in the wheel-mesh tests, whose hub row couples to every
    part.)"""
    m = BJ_MESHES[mesh]()
    rng = np.random.default_rng(12)
    wl = W.Workload("t", m, rng.uniform(0, 10, m.n_nodes), 0, None, 1.0, False, 1e-12, 0)
    T = eg().Tensor.from_mesh(m, 0)
    p = gpu_problem(T, wl)
    po = O.build_problem(wl)
    u = rng.uniform(0, 1, T.n)
    u[po.dirichlet] = 0
    jv = T.problem_jacobian(p, dt(u))
    Jo = O.jacobian(po, u)
    A = (Jo.T if transpose else Jo).tocsc()
    rhs = rng.uniform(-1, 1, T.n)
    xo = spla.spsolve(A, rhs)
    cond = np.linalg.cond(A.toarray())
    iters = {}
    for blocks, threads in ((0, 0), (7, 1024), (64, 256), (33, 512), (2, 512)):
        if blocks and (T.n + blocks - 1) // blocks > 1024:
            continue
        for pc in sorted({0, precond}):
            print(f"bicgstab block-Jacobi mesh={mesh} transpose={transpose} precond={pc} kernel={kernel} "
                  f"grid={blocks}x{threads}", flush=True)
            T.set_shape(krylov_precond=pc, krylov_blocks=blocks, krylov_threads=threads, krylov_kernel=kernel)
            x, rc, its, rr = T.solve(jv, dt(rhs), transpose=transpose, rtol=1e-12)
            assert rc == 0, (rc, its, rr)
            # the recursive residual reaches 1e-12; the true one differs from it by
            # the residual gap, of order eps cond(A)
            res = relerr(A @ host(x), rhs)
            assert res < max(5e-12, 2e-16 * cond)
            assert relerr(host(x), xo) < cond * max(res, 1e-12) * 10
            iters[(blocks, pc)] = its
            # deterministic for a fixed grid
            x2, _, its2, _ = T.solve(jv, dt(rhs), transpose=transpose, rtol=1e-12)
            assert its2 == its and torch.equal(x, x2)
    if precond >= 8 and mesh != "1d_n120":
        assert iters[(0, precond)] < iters[(0, 0)]


COARSE_REMOVED = "coarse correction removed: not faster than block-Jacobi alone (~480 us setup per solve), and its first parity case (1D, 2 parts, 1024-thread workgroups) faulted the GPU with the cause not found"


@pytest.mark.skip(reason=COARSE_REMOVED)
@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("mesh", list(BJ_MESHES))
def test_bicgstab_coarse_correction(mesh, transpose):
    """BiCGStab with the two-level preconditioner (block-Jacobi plus a coarse
    correction with one unknown per part, A_c = R^T J R inverted in every
    workgroup's LDS) against SuperLU, on grids of up to 128 parts;
    deterministic; fewer iterations than the block part alone."""
    m = BJ_MESHES[mesh]()
    rng = np.random.default_rng(16)
    wl = W.Workload("t", m, rng.uniform(0, 10, m.n_nodes), 0, None, 1.0, False, 1e-12, 0)
    T = eg().Tensor.from_mesh(m, 0)
    p = gpu_problem(T, wl)
    po = O.build_problem(wl)
    u = rng.uniform(0, 1, T.n)
    u[po.dirichlet] = 0
    jv = T.problem_jacobian(p, dt(u))
    A = (O.jacobian(po, u).T if transpose else O.jacobian(po, u)).tocsc()
    rhs = rng.uniform(-1, 1, T.n)
    xo = spla.spsolve(A, rhs)
    cond = np.linalg.cond(A.toarray())
    iters = {}
    for blocks, threads in ((0, 0), (7, 1024), (33, 512), (64, 256), (128, 1024)):
        if blocks and (T.n + blocks - 1) // blocks > threads:
            continue
        for coarse in (0, 1):
            print(f"bicgstab coarse={coarse} mesh={mesh} transpose={transpose} grid={blocks}x{threads}", flush=True)
            T.set_shape(krylov_precond=8, krylov_coarse=coarse, krylov_blocks=blocks, krylov_threads=threads)
            x, rc, its, rr = T.solve(jv, dt(rhs), transpose=transpose, rtol=1e-12)
            assert rc == 0, (rc, its, rr)
            res = relerr(A @ host(x), rhs)
            assert res < max(5e-12, 2e-16 * cond)
            assert relerr(host(x), xo) < cond * max(res, 1e-12) * 10
            iters[(blocks, coarse)] = its
            x2, _, its2, _ = T.solve(jv, dt(rhs), transpose=transpose, rtol=1e-12)
            assert its2 == its and torch.equal(x, x2)
    # the coarse space pays on the 2D grid; on the small disk (27 parts of ~60
    # rows) the block part alone already needs few iterations
    if mesh == "2d_jitter_n45":
        assert iters[(0, 1)] < iters[(0, 0)]


@pytest.mark.skip(reason=COARSE_REMOVED)
def test_newton_coarse_correction_stats():
    """Newton with the coarse correction: the oracle's solution, statistics
    bit 3 set, and 2D-256 at 128 parts fewer BiCGStab iterations than the
    block part alone."""
    wl = W.nonlinear_diffusion_2d(40, seed=78)
    T = eg().Tensor.from_mesh(wl.mesh, wl.form)
    T.set_shape(krylov_coarse=1)
    p = gpu_problem(T, wl)
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st = T.newton(p, u, _tight(), warn=False)
    assert st.status in (0, 4), st.status_name
    assert st.krylov_kernels == 13
    uo, _ = O.newton(O.build_problem(wl), tol=1e-14, max_iter=30)
    assert relerr(host(u), uo) <= 1e-10
    wl = W.nonlinear_diffusion_2d(256)
    T = eg().Tensor.from_mesh(wl.mesh, wl.form)
    p = gpu_problem(T, wl)
    its = {}
    sols = {}
    for coarse in (0, 1):
        print(f"newton 2d_256 coarse={coarse} grid=128x1024", flush=True)
        T.set_shape(krylov_coarse=coarse, krylov_blocks=128, krylov_threads=1024)
        u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
        st = T.newton(p, u, eg().NewtonOptions(tol=1e-10, forcing=1), warn=False)
        assert st.status == 0, st.status_name
        assert st.krylov_kernels == (13 if coarse else 5)
        its[coarse] = st.krylov_iters
        sols[coarse] = host(u)
    assert its[1] < its[0]
    assert relerr(sols[1], sols[0]) < 1e-8


@pytest.mark.parametrize("kernel", [0, 2])
@pytest.mark.parametrize("precond", [0, 8, 32])
@pytest.mark.parametrize("mesh", list(BJ_MESHES))
def test_cg_block_preconditioner(mesh, precond, kernel):
    """Conjugate gradients with the block-Jacobi preconditioner (symmetric
    positive definite for the SPD matrix DF(0) = K with identity Dirichlet
    rows) against SuperLU, on several grids; deterministic; fewer iterations
    than Jacobi."""
    m = BJ_MESHES[mesh]()
    rng = np.random.default_rng(14)
    wl = W.Workload("t", m, rng.uniform(0, 10, m.n_nodes), 0, None, 1.0, False, 1e-12, 0)
    T = eg().Tensor.from_mesh(m, 0)
    p = gpu_problem(T, wl)
    po = O.build_problem(wl)
    zero = np.zeros(T.n)
    jv = T.problem_jacobian(p, dt(zero))
    A = O.jacobian(po, zero).tocsc()
    assert abs(A - A.T).max() == 0.0
    rhs = rng.uniform(-1, 1, T.n)
    xo = spla.spsolve(A, rhs)
    cond = np.linalg.cond(A.toarray())
    iters = {}
    for blocks, threads in ((0, 0), (7, 1024), (64, 256), (33, 512), (2, 512)):
        if blocks and (T.n + blocks - 1) // blocks > 1024:
            continue
        for pc in sorted({0, precond}):
            print(f"cg block-Jacobi mesh={mesh} precond={pc} kernel={kernel} grid={blocks}x{threads}", flush=True)
            T.set_shape(krylov_precond=pc, krylov_blocks=blocks, krylov_threads=threads, krylov_kernel=kernel)
            x, st, its, rr = T.solve_cg(jv, dt(rhs), rtol=1e-12)
            assert st == 0, (st, its, rr)
            res = relerr(A @ host(x), rhs)
            assert res < max(5e-12, 2e-16 * cond)
            assert relerr(host(x), xo) < cond * max(res, 1e-12) * 10
            iters[(blocks, pc)] = its
            x2, _, its2, _ = T.solve_cg(jv, dt(rhs), rtol=1e-12)
            assert its2 == its and torch.equal(x, x2)
    # CG on rows wider than 8 entries (3D) runs the streaming kernel with Jacobi
    if precond >= 8 and mesh not in ("1d_n120", "3d_n9"):
        assert iters[(0, precond)] < iters[(0, 0)]


def test_block_preconditioner_shape_validation():
    T = eg().Tensor.from_mesh(W.mesh_2d(6), 0)
    assert T.get_shape()["krylov_precond"] == 8
    for bad in (-1, 1, 33):
        with pytest.raises(eg().EgfemError):
            T.set_shape(krylov_precond=bad)
    T.set_shape(krylov_precond=2)
    assert T.get_shape()["krylov_precond"] == 2
    # the Chebyshev interval ratio: [2, 1000], 0 = the default 30
    assert T.get_shape()["krylov_cheb_ratio"] == 30.0
    for bad in (1.5, -1.0, 2000.0, float("nan")):
        with pytest.raises(eg().EgfemError):
            T.set_shape(krylov_cheb_ratio=bad)
    T.set_shape(krylov_cheb_ratio=20.0)
    assert T.get_shape()["krylov_cheb_ratio"] == 20.0
    T.set_shape(krylov_cheb_ratio=0.0)
    assert T.get_shape()["krylov_cheb_ratio"] == 30.0


@pytest.mark.parametrize("ratio", [10.0, 20.0, 50.0, 200.0])
def test_cheb_ratio_solves_to_oracle(ratio):
    """Every Chebyshev interval ratio gives a fixed linear block preconditioner:
    the overlapped and barrier-form BiCGStab solve the Newton systems to the
    oracle's solution."""
    wl = W.nonlinear_diffusion_2d(40, seed=71)
    T = eg().Tensor.from_mesh(wl.mesh, wl.form)
    p = gpu_problem(T, wl)
    uo, _ = O.newton(O.build_problem(wl), tol=1e-14, max_iter=40)
    for kernel in (0, 2):
        T.set_shape(krylov_cheb_ratio=ratio, krylov_kernel=kernel)
        u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
        st = T.newton(p, u, eg().NewtonOptions(tol=1e-13, krylov_rtol=1e-13), warn=False)
        assert st.status in (0, 4) and st.krylov_kernels & 4, (st.status_name, st.krylov_kernels)
        assert relerr(host(u), uo) < 1e-10


# ---------------------------------------------------------------------------
# Newton
# ---------------------------------------------------------------------------
def _tight():
    return eg().NewtonOptions(tol=1e-14, max_newton=30, krylov_rtol=1e-14)


@pytest.mark.parametrize("name", ["1d", "2d_n40", "2d_semilinear_n33", "3d_kappa_n6"])
def test_newton_matches_oracle(name):
    wl = WORKLOADS_SMALL[name]()
    T = eg().Tensor.from_mesh(wl.mesh, wl.form)
    p = gpu_problem(T, wl)
    po = O.build_problem(wl)
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st = T.newton(p, u, _tight(), warn=False)
    assert st.status in (0, 4), st.status_name
    uo, sto = O.newton(po, tol=1e-14, max_iter=30)
    ug = host(u)
    assert relerr(ug, uo) <= 1e-10
    # certificate: the oracle's residual at the GPU solution
    Fo0 = np.linalg.norm(po.d[~po.dirichlet])
    assert np.linalg.norm(O.residual(po, ug)) <= 1e-11 * Fo0


@pytest.mark.parametrize("kernel,precond", [(0, 8), (0, 0), (1, 8), (2, 8)])
def test_newton_krylov_kernels(kernel, precond):
    """The register-resident BiCGStab (block-Jacobi in its overlapped form or
    in the barrier form, or Jacobi) and the streaming one (always Jacobi) give
    the oracle's solution, and the statistics name the kernel that ran (bit 2:
    block preconditioner, bit 3: overlapped form)."""
    wl = W.nonlinear_diffusion_2d(40, seed=77)
    T = eg().Tensor.from_mesh(wl.mesh, wl.form)
    T.set_shape(krylov_kernel=kernel, krylov_precond=precond)
    p = gpu_problem(T, wl)
    po = O.build_problem(wl)
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st = T.newton(p, u, _tight(), warn=False)
    assert st.status in (0, 4), st.status_name
    want = {(0, 8): 13, (0, 0): 1, (1, 8): 2, (2, 8): 5}[(kernel, precond)]
    assert st.krylov_kernels == want
    uo, _ = O.newton(po, tol=1e-14, max_iter=30)
    assert relerr(host(u), uo) <= 1e-10


def test_newton_full_size_2d_256():
    """The 2D nonlinear-diffusion workload at full size (66,049 nodes)."""
    wl = W.nonlinear_diffusion_2d(256)
    T = eg().Tensor.from_mesh(wl.mesh, wl.form)
    p = gpu_problem(T, wl)
    po = O.build_problem(wl)
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st = T.newton(p, u, _tight(), warn=False)
    assert st.status in (0, 4), st.status_name
    uo, _ = O.newton(po, tol=1e-14, max_iter=30)
    ug = host(u)
    assert relerr(ug, uo) <= 1e-10
    assert np.linalg.norm(O.residual(po, ug)) <= 1e-10 * np.linalg.norm(po.d[~po.dirichlet])
    # the performance configuration (Eisenstat-Walker forcing, tol 1e-10)
    u2 = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st2 = T.newton(p, u2, eg().NewtonOptions(tol=1e-10, forcing=1), warn=False)
    assert st2.status == 0
    assert st2.res <= 1e-10 * st2.res0
    # per-step Krylov diagnostics: every accepted step had a converged linear
    # solve that reduced the residual (forcing terms are below one)
    k = st2.newton_iters
    assert len(st2.krylov_status_hist) == min(k + 1, 64) and len(st2.krylov_hist) == k
    assert all(s == 0 for s in st2.krylov_status_hist[:k])
    assert all(0.0 < r < 1.0 for r in st2.krylov_relres_hist[:k])
    assert np.linalg.norm(O.residual(po, host(u2))) <= 1.01e-10 * np.linalg.norm(po.d[~po.dirichlet])


def test_newton_deterministic():
    wl = W.nonlinear_diffusion_2d(64)
    T = eg().Tensor.from_mesh(wl.mesh, wl.form)
    p = gpu_problem(T, wl)
    outs = []
    for _ in range(2):
        u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
        T.newton(p, u, eg().NewtonOptions(tol=1e-10, forcing=1))
        outs.append(host(u))
    assert np.array_equal(outs[0], outs[1])


def test_newton_edge_cases():
    E = eg()
    # one interior node: 4u + 2u^3 = d_1
    wl = W.Workload("t", W.mesh_1d(2), np.full(3, 7.0), 0, None, 1.0, False, 1e-14, 0)
    T = E.Tensor.from_mesh(wl.mesh, 0)
    p = gpu_problem(T, wl)
    u = torch.zeros(3, dtype=torch.float64, device=DEV)
    st = T.newton(p, u, _tight(), warn=False)
    d1 = host(p.load)[1]
    ug = host(u)
    assert abs(4 * ug[1] + 2 * ug[1] ** 3 - d1) <= 1e-13 * abs(d1)
    assert ug[0] == 0.0 and ug[2] == 0.0
    # zero load: u = 0 at once
    wl0 = W.Workload("t", W.mesh_2d(5), np.zeros(36), 0, None, 1.0, False, 1e-12, 0)
    T0 = E.Tensor.from_mesh(wl0.mesh, 0)
    u0 = torch.zeros(36, dtype=torch.float64, device=DEV)
    st0 = T0.newton(gpu_problem(T0, wl0), u0)
    assert st0.status == 0 and st0.newton_iters == 0 and not host(u0).any()
    # warm start at the solution: the iterate does not move
    u1 = u.clone()
    st1 = T.newton(p, u1, E.NewtonOptions(tol=1e-12), warn=False)
    assert st1.status in (0, 4)
    assert np.abs(host(u1) - ug).max() <= 1e-14 * np.abs(ug).max()
    # NaN in the initial guess -> nonfinite status, no exception
    un = torch.full((3,), float("nan"), dtype=torch.float64, device=DEV)
    stn = T.newton(p, un, warn=False)
    assert stn.status_name == "nonfinite"
    # iteration cap
    wl2 = W.nonlinear_diffusion_2d(24)
    T2 = E.Tensor.from_mesh(wl2.mesh, 0)
    u2 = torch.zeros(T2.n, dtype=torch.float64, device=DEV)
    st2 = T2.newton(gpu_problem(T2, wl2), u2, E.NewtonOptions(max_newton=1), warn=False)
    assert st2.status_name == "not_converged" and st2.newton_iters == 1


# ---------------------------------------------------------------------------
# full-size spot checks (rows the oracle assembles one by one)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["2d_semilinear_512", "3d_64"])
def test_full_size_sampled_rows(which):
    wl = W.semilinear_2d(512) if which == "2d_semilinear_512" else W.diffusion_3d(64)
    m = wl.mesh
    T = eg().Tensor.from_mesh(m, wl.form)
    rng = np.random.default_rng(12)
    rows = np.unique(np.concatenate([rng.integers(0, m.n_nodes, 300), [0, m.n_nodes - 1,
                                                                       m.n_nodes // 2]]))
    u = rng.uniform(-1, 1, m.n_nodes)
    a = rng.uniform(0.5, 2, m.n_nodes)
    g = rng.uniform(-2, 2, m.n_nodes)
    Tr = O.tensor_rows(m.coords, m.cells, wl.form, rows)
    r = host(T.residual(dt(u), dt(a)))
    ro = O.contract_uv(Tr, u, a)
    assert relerr(r[rows], ro[rows]) < 1e-12
    Jg = csr_of(T, T.jacobian(dt(u), dt(a), dt(g)))
    Jo = (O.contract_first(Tr, a) + O.contract_mode2(Tr, u) @ sp.diags(g)).tocsr()
    d = (Jg[rows] - Jo[rows])
    assert abs(d).max() <= 1e-12 * abs(Jo[rows]).max()


@pytest.mark.parametrize("form", [1, 2])
@pytest.mark.parametrize("mesh", ["1d_n257", "2d_n37", "2d_jitter_n21", "3d_n7"])
def test_symmetric_half_stream(mesh, form):
    """Tensors with T_ijk = T_ikj: the half-stream action equals the full
    stream's and the oracle's, raw and in the problem residual."""
    m = MESHES[mesh]()
    T = eg().Tensor.from_mesh(m, form)
    assert T.info.nnz_half > 0 and T.get_shape()["action_half"] == 0
    T.set_shape(action_half=1)
    To = O.assemble_tensor(m.coords, m.cells, form)
    rng = np.random.default_rng(41)
    u = rng.uniform(-1, 1, m.n_nodes)
    a = rng.uniform(0.5, 2, m.n_nodes)
    rh = host(T.residual(dt(u), dt(a)))
    T.set_shape(action_half=0)
    rf = host(T.residual(dt(u), dt(a)))
    assert relerr(rh, O.contract_uv(To, u, a)) < 1e-12
    assert np.abs(rh - rf).max() <= 1e-13 * np.abs(rf).max()
    # problem residual (semilinear form: K u + T:(u (x) u^2) - d) with both streams
    wl = W.Workload("t", m, rng.uniform(-5, 5, m.n_nodes), form, None, 0.0, True, 1e-10, 1)
    p = gpu_problem(T, wl)
    Ff = host(T.problem_residual(p, dt(u)))
    T.set_shape(action_half=1)
    Fh = host(T.problem_residual(p, dt(u)))
    po = O.build_problem(wl)
    assert relerr(Fh, O.residual(po, u)) < 1e-12
    assert np.abs(Fh - Ff).max() <= 1e-13 * np.abs(Ff).max()
    # a stiffness tensor has no half stream
    S = eg().Tensor.from_mesh(m, 0)
    assert S.get_shape()["action_half"] == 0
    with pytest.raises(eg().EgfemError):
        S.set_shape(action_half=1)


def test_newton_full_size_semilinear_512():
    """The 2D 512x512 semilinear workload (mass tensor plus K, 263,169 nodes):
    the GPU Newton solution against the oracle's, both to a 1e-12 residual."""
    print("newton full size 2d semilinear 512", flush=True)
    wl = W.semilinear_2d(512)
    T = eg().Tensor.from_mesh(wl.mesh, wl.form)
    p = gpu_problem(T, wl)
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st = T.newton(p, u, eg().NewtonOptions(tol=1e-12, krylov_rtol=1e-13), warn=False)
    assert st.status in (0, 4), st.status_name
    # 263,169 rows exceed one row per thread of the 256/512-thread resident
    # grids; the 261,121 free rows fit 1024-thread workgroups: resident
    # block-Jacobi BiCGStab on the free-row partition
    assert st.krylov_kernels == 5, st.krylov_kernels
    po = O.build_problem(wl)
    uo, sto = O.newton(po, tol=1e-12)
    ug = host(u)
    assert relerr(ug, uo) < 1e-10
    assert np.linalg.norm(O.residual(po, ug)) <= 1e-11 * np.linalg.norm(po.d[po.free])


def test_newton_full_size_3d_64_certificate():
    """The 3D 64^3 workload (274,625 nodes) in the benchmark configuration (EW
    forcing, 1e-10): the residual the oracle computes on sampled rows (tensor rows
    assembled one by one) at the GPU solution is within the global tolerance."""
    print("newton full size 3d 64", flush=True)
    wl = W.diffusion_3d(64)
    m = wl.mesh
    T = eg().Tensor.from_mesh(m, wl.form)
    p = gpu_problem(T, wl)
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st = T.newton(p, u, eg().NewtonOptions(tol=1e-10, forcing=1))
    assert st.status == 0 and st.res <= 1e-10 * st.res0
    ug = host(u)
    rng = np.random.default_rng(77)
    rows = np.unique(rng.integers(0, m.n_nodes, 400))
    rows = rows[m.dirichlet[rows] == 0]
    Tr = O.tensor_rows(m.coords, m.cells, wl.form, rows)
    b = O.assemble_mass(m.coords, m.cells) @ wl.f
    F = O.contract_uv(Tr, ug, wl.a0 + ug * ug) - b
    free = m.dirichlet == 0
    assert np.abs(F[rows]).max() <= 2e-10 * np.linalg.norm(b[free])
    # and the GPU's own residual on those rows agrees with the oracle's
    Fg = host(T.problem_residual(p, u))
    assert np.abs(Fg[rows] - F[rows]).max() <= 1e-12 * np.abs(b).max()


@pytest.mark.parametrize("kernel", [0, 1, 2])
def test_newton_timing_leaves_the_iteration_unchanged(kernel):
    """Each Newton step enqueues its trial residual behind the Krylov launch and
    reads the solve's outcome, timing events and the trial norm in one
    synchronisation: with timing on, the iterate and the per-step statistics
    are bitwise the untimed ones, and every stage's time is reported."""
    wl = W.nonlinear_diffusion_2d(40, seed=57)
    T = eg().Tensor.from_mesh(wl.mesh, wl.form)
    T.set_shape(krylov_kernel=kernel)
    p = gpu_problem(T, wl)
    runs = []
    for timing in (0, 1, 0):
        u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
        st = T.newton(p, u, eg().NewtonOptions(tol=1e-10, forcing=1, timing=timing))
        assert st.status == 0, st.status_name
        assert st.newton_iters <= 64 and sum(st.krylov_hist) == st.krylov_iters
        assert (st.t_krylov_ms > 0.0) == bool(timing)
        assert (st.t_action_ms > 0.0 and st.t_jacobian_ms > 0.0) == bool(timing)
        runs.append((u, st))
    (u0, s0), (u1, s1), (u2, s2) = runs
    assert torch.equal(u0, u1) and torch.equal(u0, u2)
    assert s0.krylov_hist == s1.krylov_hist == s2.krylov_hist
    assert s0.res_hist == s1.res_hist and s0.backtracks == s1.backtracks
    un, _ = O.newton(O.build_problem(wl), tol=1e-14)
    assert relerr(host(u1), un) <= 1e-8


# ---------------------------------------------------------------------------
# free-row resident BiCGStab (1024-thread workgroups, Dirichlet rows left out)
# ---------------------------------------------------------------------------
FREE_ROW_CASES = {
    "2d_n96": lambda: W.nonlinear_diffusion_2d(96, seed=61),
    "2d_semilinear_n64": lambda: W.semilinear_2d(64),
    "1d_n3000": lambda: W.nonlinear_diffusion_1d(3000),
    # 3D Kuhn rows hold up to 15 entries: 8 in registers, the rest in LDS
    "3d_kappa_n12": lambda: W.diffusion_3d(12),
    "3d_kappa_n17": lambda: W.diffusion_3d(17),
}


@pytest.mark.parametrize("name", list(FREE_ROW_CASES))
def test_newton_free_rows_matches_oracle(name):
    """Newton with 1024-thread Krylov workgroups: the Dirichlet rows (identity
    rows, zero residual) are left out of the resident block-Jacobi BiCGStab,
    which runs on a compact partition of the free rows; the solution equals
    the oracle's element-wise, as with the default grid."""
    wl = FREE_ROW_CASES[name]()
    print(f"newton free rows {name}", flush=True)
    T = eg().Tensor.from_mesh(wl.mesh, wl.form)
    p = gpu_problem(T, wl)
    opts = eg().NewtonOptions(tol=1e-13, krylov_rtol=1e-13)
    uo, _ = O.newton(O.build_problem(wl), tol=1e-14, max_iter=40)
    for kernel in (0, 2):     # both select the barrier form at 1024 threads
        T.set_shape(krylov_threads=1024, krylov_blocks=0, krylov_kernel=kernel)
        u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
        st = T.newton(p, u, opts, warn=False)
        assert st.status in (0, 4), st.status_name
        assert st.krylov_kernels == 5, st.krylov_kernels
        ug = host(u)
        assert relerr(ug, uo) < 1e-10
        assert np.abs(ug - uo).max() <= 1e-10 * np.abs(uo).max()
        assert np.all(ug[wl.mesh.dirichlet != 0] == 0.0)
        # deterministic
        u2 = torch.zeros(T.n, dtype=torch.float64, device=DEV)
        st2 = T.newton(p, u2, opts, warn=False)
        assert torch.equal(u, u2) and st2.krylov_iters == st.krylov_iters


@pytest.mark.parametrize("n", [5, 10, 22])
def test_newton_wide_rows_default_shape(n):
    """3D meshes (rows of up to 15 entries) with the default launch shape: the
    solve runs the 1024-thread resident block-Jacobi BiCGStab on the free
    rows (one part for n = 5 and 10, several for n = 22: 9,261 free rows) and
    equals the oracle's solution element-wise."""
    wl = W.diffusion_3d(n)
    print(f"newton wide rows default shape n={n}", flush=True)
    T = eg().Tensor.from_mesh(wl.mesh, wl.form)
    rowptr = np.asarray(T.pattern()[0])
    assert np.diff(rowptr).max() == 15
    p = gpu_problem(T, wl)
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st = T.newton(p, u, eg().NewtonOptions(tol=1e-13, krylov_rtol=1e-13), warn=False)
    assert st.status in (0, 4), st.status_name
    assert st.krylov_kernels == 5, st.krylov_kernels
    uo, _ = O.newton(O.build_problem(wl), tol=1e-14, max_iter=40)
    ug = host(u)
    assert relerr(ug, uo) < 1e-10
    assert np.abs(ug - uo).max() <= 1e-10 * np.abs(uo).max()
    assert np.all(ug[wl.mesh.dirichlet != 0] == 0.0)


def test_newton_free_rows_mask_change_rebuilds_partition():
    """The same handle solved with two different Dirichlet sets (the whole
    boundary, then only the left and right walls, in one buffer rewritten in
    place): the free-row partition follows the mask and both solutions equal
    the oracle's."""
    E = eg()
    wl = W.nonlinear_diffusion_2d(64, seed=62)
    m = wl.mesh
    T = E.Tensor.from_mesh(m, wl.form)
    T.set_shape(krylov_threads=1024, krylov_blocks=0)
    load = T.matvec(dt(wl.f), "M")
    mask = dt(m.dirichlet, torch.uint8)
    p = E.Problem(T.n, load, mask, None, wl.a0_const, wl.add_stiffness)
    x = np.asarray(m.coords)[:, 0]
    walls = ((x <= 1e-12) | (x >= 1 - 1e-12)).astype(np.uint8)
    for dmask in (np.asarray(m.dirichlet, np.uint8), walls):
        mask.copy_(dt(dmask, torch.uint8))
        u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
        st = T.newton(p, u, E.NewtonOptions(tol=1e-13, krylov_rtol=1e-13), warn=False)
        assert st.status in (0, 4) and st.krylov_kernels == 5, (st.status_name, st.krylov_kernels)
        wlm = W.Workload(wl.name, W.Mesh(m.dim, m.n, m.coords, m.cells, dmask), wl.f, wl.form, wl.a0,
                         wl.a0_const, wl.add_stiffness, wl.tol, wl.seed)
        po = O.build_problem(wlm)
        uo, _ = O.newton(po, tol=1e-14, max_iter=40)
        assert relerr(host(u), uo) < 1e-10
