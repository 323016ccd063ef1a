"""Launch-shape autotuner: every candidate shape of the tensor action gives
bitwise identical results (the per-row summation order does not depend on
the shape), and a tuned handle still solves to the oracle's solution."""
import numpy as np
import pytest
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


@pytest.mark.parametrize("wlname", ["2d_n96", "3d_n12", "semilinear_n64"])
def test_action_shapes_bitwise_equal(wlname):
    wl = {"2d_n96": lambda: W.nonlinear_diffusion_2d(96), "3d_n12": lambda: W.diffusion_3d(12),
          "semilinear_n64": lambda: W.semilinear_2d(64)}[wlname]()
    T = eg().Tensor.from_mesh(wl.mesh, wl.form)
    rng = np.random.default_rng(3)
    u = dt(rng.uniform(-1, 1, T.n))
    a = dt(rng.uniform(0.5, 2, T.n))
    load = T.matvec(dt(wl.f), "M")
    p = eg().Problem(T.n, load, dt(wl.mesh.dirichlet, torch.uint8), dt(wl.a0) if wl.a0 is not None else None,
                     wl.a0_const, wl.add_stiffness)
    T.set_shape(action_runs=0, action_pipe=0)
    ref = host(T.residual(u, a))
    Fref, nref = T.problem_residual(p, u, with_norm=True)
    Fref = host(Fref)
    nb = T.info.row_blocks
    for runs, pipe in ((0, 0), (max(1, nb // 3), 0), (max(1, nb // 3), 1), (max(1, nb // 7), 1), (1, 1),
                       (nb + 5, 0)):
        T.set_shape(action_runs=runs, action_pipe=pipe)
        assert np.array_equal(host(T.residual(u, a)), ref), (runs, pipe)
        F, nF = T.problem_residual(p, u, with_norm=True)
        assert np.array_equal(host(F), Fref), (runs, pipe)
        assert abs(nF - nref) <= 1e-14 * nref   # partial sums regroup with the run count
    To = O.assemble_tensor(wl.mesh.coords, wl.mesh.cells, wl.form)
    r = O.contract_uv(To, host(u), host(a))
    assert np.linalg.norm(ref - r) <= 1e-12 * np.linalg.norm(r)


def test_autotuned_handle_solves():
    E = eg()
    wl = W.nonlinear_diffusion_2d(64)
    T = E.Tensor.from_mesh(wl.mesh, wl.form)
    load = T.matvec(dt(wl.f), "M")
    p = E.Problem(T.n, load, dt(wl.mesh.dirichlet, torch.uint8), None, 1.0, False)
    res = T.autotune(p)
    s = res["shape"]
    assert s["action_pipe"] in (0, 1) and s["krylov_threads"] in (256, 512, 1024)
    # the block preconditioner's steps and interval come from the tuner's candidates
    assert s["krylov_precond"] in (6, 8, 10) and s["krylov_cheb_ratio"] in (20.0, 30.0, 50.0)
    assert res["action_us"] > 0 and res["krylov_iter_us"] > 0
    assert T.get_shape() == s
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    st = T.newton(p, u, E.NewtonOptions(tol=1e-14, krylov_rtol=1e-14, max_newton=40), warn=False)
    assert st.status in (0, 4)
    uo, _ = O.newton(O.build_problem(wl), tol=1e-14, max_iter=40)
    assert np.linalg.norm(host(u) - uo) <= 1e-10 * np.linalg.norm(uo)
    with pytest.raises(E.EgfemError):
        T.set_shape(krylov_threads=300)
