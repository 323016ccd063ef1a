"""egfem_problem_residual_noalloc (the entry point for callers that cannot
allocate) against egfem_problem_residual on the same inputs: F bitwise, the
norm to 1e-14 (another fixed summation order), on two calls in a row with the
second on a smaller input, including the oracle's residual as a check of
both; a handle whose residual kernel writes more partial sums than the fixed
array holds is rejected with EGFEM_ERR_SHAPE."""
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


def setup(wl):
    E = eg()
    T = E.Tensor.from_mesh(wl.mesh, wl.form)
    load = T.matvec(torch.tensor(wl.f, dtype=torch.float64, device=DEV), "M")
    dirm = torch.tensor(wl.mesh.dirichlet, dtype=torch.uint8, device=DEV)
    a0 = torch.tensor(wl.a0, dtype=torch.float64, device=DEV) if wl.a0 is not None else None
    return T, E.Problem(T.n, load, dirm, a0, wl.a0_const, wl.add_stiffness)


def test_noalloc_residual_matches_allocating_entry_point():
    # the larger input first, then a smaller one: the second call must not see
    # the first call's partial sums
    cases = [W.semilinear_2d(96), W.nonlinear_diffusion_2d(24)]
    for wl in cases:
        print(f"noalloc residual {wl.name} nodes={wl.mesh.n_nodes}", flush=True)
        T, p = setup(wl)
        rng = np.random.default_rng(3)
        u0 = rng.uniform(-1, 1, T.n)
        u0[np.asarray(wl.mesh.dirichlet, bool)] = 0.0
        u = torch.tensor(u0, dtype=torch.float64, device=DEV)
        F_ref, n_ref = T.problem_residual(p, u, with_norm=True)
        F = torch.full_like(u, float("nan"))
        F_na, n_na = T.problem_residual_noalloc(p, u, F, with_norm=True)
        torch.cuda.synchronize()
        assert torch.equal(F_na, F_ref)
        assert abs(n_na - n_ref) <= 1e-14 * n_ref
        Fo = O.residual(O.build_problem(wl), u0)
        assert abs(n_na - np.linalg.norm(Fo)) <= 1e-12 * np.linalg.norm(Fo)
        # without the norm: F only
        F2 = torch.zeros_like(u)
        T.problem_residual_noalloc(p, u, F2)
        torch.cuda.synchronize()
        assert torch.equal(F2, F_ref)
        T.close()


def test_noalloc_residual_rejects_too_many_partials():
    E = eg()
    wl = W.diffusion_3d(64)           # 16,832 row blocks: one partial sum each when untuned
    T, p = setup(wl)
    assert T.info.row_blocks > 16384
    u = torch.zeros(T.n, dtype=torch.float64, device=DEV)
    F = torch.empty_like(u)
    with pytest.raises(E.EgfemError) as ei:
        T.problem_residual_noalloc(p, u, F, with_norm=True)
    assert ei.value.code == -2          # EGFEM_ERR_SHAPE
    # with action runs below the limit the same handle is accepted
    T.set_shape(action_runs=8192)
    F_na, n_na = T.problem_residual_noalloc(p, u, F, with_norm=True)
    F_ref, n_ref = T.problem_residual(p, u, with_norm=True)
    torch.cuda.synchronize()
    assert torch.equal(F_na, F_ref) and abs(n_na - n_ref) <= 1e-14 * n_ref
    T.close()
