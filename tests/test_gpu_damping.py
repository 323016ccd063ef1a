"""The damping rule of the Newton iteration (remark at the end of Sec. 4) on
the GPU drivers: the host-driven egfem_newton and the device line search of
the batched persistent launch.  One free node, F(u) = 4u + 2u^3 - d1, where
the oracle's hand-checked pins fix every trial: f = -12 halves the first step
once (u1 = -0.75, |F| = 2.15625, then the root u = -1); d1^2 = 31.999 is
rejected by the sufficient-decrease constant 1e-4 although |F| falls, and
d1^2 = 32 (1 - 1.5e-4) is accepted at full step."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import egfem_oracle as O

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# (nodal f, backtracks of step 1, u after step 1 as a multiple of d1)
CASES = [(-12.0, 1, 0.125), (2.0 * -math.sqrt(31.999), 1, 0.125),
         (2.0 * -math.sqrt(32.0 * (1.0 - 1.5e-4)), 0, 0.25)]


def eg():
    import paper_2005_06193_amd as mod
    return mod


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def one_node(fval):
    E = eg()
    wl = W.Workload("t", W.mesh_1d(2), np.full(3, fval), 0, None, 1.0, False, 1e-14, 0)
    T = E.Tensor.from_mesh(wl.mesh, 0)
    f = torch.tensor(wl.f, dtype=torch.float64, device=DEV)
    load = T.matvec(f, "M")
    dirm = torch.tensor(wl.mesh.dirichlet, dtype=torch.uint8, device=DEV)
    return wl, T, E.Problem(T.n, load, dirm, None, 1.0, False)


def opts(max_newton, tol=1e-15):
    return eg().NewtonOptions(tol=tol, max_newton=max_newton, krylov_rtol=1e-15)


def check_first_step(wl, st, u, back, frac):
    po = O.build_problem(wl)
    uo, so = O.newton(po, tol=1e-15, max_iter=1)
    d1 = po.d[1]
    assert st.newton_iters == 1
    assert st.backtracks == back == so.backtracks
    ug = host(u)
    assert abs(ug[1] - frac * d1) <= 1e-14 * abs(d1)   # d1/8 after one halving, d1/4 at full step
    assert abs(ug[1] - uo[1]) <= 1e-14 * abs(uo[1])
    assert abs(st.res_hist[0] - so.residual_norms[1]) <= 1e-13 * so.residual_norms[1]
    assert abs(st.res0 - so.residual_norms[0]) <= 1e-14 * so.residual_norms[0]


def check_solution(wl, st, u):
    po = O.build_problem(wl)
    # tolerance above the rounding floor: both sides stop on the test, not by
    # stagnation (whose trials would add backtracks)
    uo, so = O.newton(po, tol=1e-13, max_iter=60)
    assert so.status == "converged"
    assert st.status == 0, st.status_name
    assert st.backtracks == so.backtracks
    ug = host(u)
    assert abs(ug[1] - uo[1]) <= 1e-14 * abs(uo[1])
    assert ug[0] == 0.0 and ug[2] == 0.0
    # residual histories agree step by step where both sides recorded one
    k = min(len(st.res_hist), len(so.residual_norms) - 1, 3)
    for a, b in zip(st.res_hist[:k], so.residual_norms[1:k + 1]):
        assert abs(a - b) <= 1e-12 * so.residual_norms[0]


@pytest.mark.parametrize("fval,back,frac", CASES)
def test_host_newton_damping(fval, back, frac):
    wl, T, p = one_node(fval)
    u = torch.zeros(3, dtype=torch.float64, device=DEV)
    st = T.newton(p, u, opts(1), warn=False)
    check_first_step(wl, st, u, back, frac)
    u = torch.zeros(3, dtype=torch.float64, device=DEV)
    st = T.newton(p, u, opts(60, 1e-13), warn=False)
    check_solution(wl, st, u)
    if fval == -12.0:
        assert abs(host(u)[1] + 1.0) <= 1e-14


def test_batched_newton_damping():
    E = eg()
    items = [one_node(f) for f, _, _ in CASES]
    Ts = [t for _, t, _ in items]
    Ps = [p for _, _, p in items]
    for max_newton, tol in ((1, 1e-15), (60, 1e-13)):
        us = [torch.zeros(3, dtype=torch.float64, device=DEV) for _ in items]
        stats, rc = E.newton_batched(Ts, Ps, us, opts(max_newton, tol))
        for (wl, _, _), (_, back, frac), st, u in zip(items, CASES, stats, us):
            if max_newton == 1:
                check_first_step(wl, st, u, back, frac)
            else:
                check_solution(wl, st, u)
