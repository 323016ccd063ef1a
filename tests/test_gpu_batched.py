"""Batched persistent Newton: every instance of one launch equals its own
per-instance solve and the oracle; hipGraph replays equal the eager run; the
64-instance workload converges."""
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


def relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def setup(wls):
    E = eg()
    Ts, Ps = [], []
    for wl in wls:
        T = E.Tensor.from_mesh(wl.mesh, wl.form)
        load = T.matvec(dt(wl.f), "M")
        a0 = dt(wl.a0) if wl.a0 is not None else None
        Ps.append(E.Problem(T.n, load, dt(wl.mesh.dirichlet, torch.uint8), a0, wl.a0_const,
                            wl.add_stiffness))
        Ts.append(T)
    return Ts, Ps


def mixed():
    return [W.nonlinear_diffusion_2d(n, seed=7 + n) for n in (5, 17, 24, 40)] + \
        [W.nonlinear_diffusion_1d(64), W.semilinear_2d(20), W.diffusion_3d(5)]


@pytest.mark.parametrize("threads", [512, 1024])
def test_batched_matches_per_instance_and_oracle(threads):
    E = eg()
    wls = mixed()
    Ts, Ps = setup(wls)
    opts = E.NewtonOptions(tol=1e-14, max_newton=40, krylov_rtol=1e-14, krylov_threads=threads)
    us = [torch.zeros(T.n, dtype=torch.float64, device=DEV) for T in Ts]
    stats, rc = E.newton_batched(Ts, Ps, us, opts)
    assert rc in (0, 4), rc
    for wl, T, P, u, st in zip(wls, Ts, Ps, us, stats):
        assert st.status in (0, 4), (wl.name, st.status_name)
        ref = torch.zeros(T.n, dtype=torch.float64, device=DEV)
        T.newton(P, ref, opts, warn=False)
        assert relerr(host(u), host(ref)) < 1e-11, wl.name
        uo, _ = O.newton(O.build_problem(wl), tol=1e-14, max_iter=40)
        ug = host(u)
        assert relerr(ug, uo) < 1e-10, wl.name
        assert np.abs(ug - uo).max() <= 1e-10 * np.abs(uo).max(), wl.name


def test_batched_graph_replays_equal_eager():
    E = eg()
    wls = [W.nonlinear_diffusion_2d(n, seed=100 + n) for n in (12, 33, 48, 64)]
    Ts, Ps = setup(wls)
    us = [torch.full((T.n,), 0.3, dtype=torch.float64, device=DEV) for T in Ts]
    B = E.Batch(Ts, Ps, us, E.NewtonOptions(tol=1e-10, forcing=1))
    B.run(zero_init=True)
    st0, rc0 = B.stats()
    assert rc0 == 0
    eager = [host(u).copy() for u in us]
    for rep in range(3):
        for u in us:
            u.fill_(float(rep + 1))          # the program's own eager work between replays
        torch.cuda.synchronize()
        B.run(zero_init=True, graph=True)
        st, rc = B.stats()
        assert rc == 0
        for e, u, s, s0 in zip(eager, us, st, st0):
            assert np.array_equal(host(u), e), rep
            assert s.newton_iters == s0.newton_iters and s.krylov_iters == s0.krylov_iters
            assert s.krylov_status_hist == s0.krylov_status_hist
            assert s.krylov_relres_hist == s0.krylov_relres_hist
    B.close()


_FULL_ORACLE = {}


def _full_oracle_problems(wls):
    """The oracle's problems of the 64-instance workload (assembled once per
    test session: both plan kinds are checked against them)."""
    if not _FULL_ORACLE:
        for m, wl in enumerate(wls):
            _FULL_ORACLE[m] = O.build_problem(wl)
    return _FULL_ORACLE


@pytest.mark.parametrize("kind", [0, 1])
def test_batched_full_workload_64_instances(kind):
    """64 instances, n ~ U{32..256}, one launch (streaming teams, kind 0, or
    scheduled resident teams, kind 1); all converge to 1e-10, each passes the
    oracle's residual test, and sampled instances' per-instance solves pass it
    too."""
    E = eg()
    print(f"batched full workload kind={kind}", flush=True)
    wls = W.nonlinear_diffusion_batch(64)
    Ts, Ps = setup(wls)
    us = [torch.zeros(T.n, dtype=torch.float64, device=DEV) for T in Ts]
    opts = E.NewtonOptions(tol=1e-10, forcing=1)
    B = E.Batch(Ts, Ps, us, opts, kind=kind)
    B.run(zero_init=True, graph=True)
    stats, rc = B.stats()
    assert rc == 0
    for s in stats:
        assert s.status == 0 and s.res <= 1e-10 * s.res0
        assert s.krylov_kernels == (5 if kind == 1 else 2)
    teams, total = B.teams()
    assert min(teams) >= 1
    if kind == 0:
        assert sum(teams) == total
    else:
        # scheduled teams reuse the resident workgroups: more team members
        # than workgroups, every team within them, one row per thread
        assert sum(teams) > total and max(teams) <= total
        for T, g in zip(Ts, teams):
            assert g * 256 >= T.n
    # every instance: the oracle's own residual at the GPU solution passes the
    # oracle's test at 1e-10 (the oracle assembles each instance's tensor)
    pos = _full_oracle_problems(wls)
    for m, wl in enumerate(wls):
        po = pos[m]
        nres = np.linalg.norm(O.residual(po, host(us[m])))
        assert nres <= 1.01e-10 * np.linalg.norm(po.d[~po.dirichlet]), (m, wl.name)
    for m in (0, 17, int(np.argmax([T.n for T in Ts]))):
        ref = torch.zeros(Ts[m].n, dtype=torch.float64, device=DEV)
        Ts[m].newton(Ps[m], ref, opts)
        po = pos[m]
        assert np.linalg.norm(O.residual(po, host(ref))) <= 1.01e-10 * np.linalg.norm(po.d[~po.dirichlet])
    B.close()


@pytest.mark.parametrize("threads", [512, 1024])
def test_batched_large_team_matches_oracle(threads):
    """A batch in which one instance is owned by a team of at least 16
    workgroups (the grouped-arrival barrier path of the team barrier) and
    smaller ones by small teams; every instance solved tightly and compared
    element-wise with the oracle's Newton solution."""
    E = eg()
    wls = [W.nonlinear_diffusion_2d(96, seed=31), W.nonlinear_diffusion_2d(12, seed=32),
           W.nonlinear_diffusion_1d(64), W.semilinear_2d(24)]
    Ts, Ps = setup(wls)
    us = [torch.zeros(T.n, dtype=torch.float64, device=DEV) for T in Ts]
    opts = E.NewtonOptions(tol=1e-14, max_newton=40, krylov_rtol=1e-14)
    B = E.Batch(Ts, Ps, us, opts, threads=threads)
    teams, total = B.teams()
    assert max(teams) >= 16 and sum(teams) == total
    B.run(zero_init=True)
    stats, rc = B.stats()
    B.close()
    assert rc in (0, 4), rc
    for wl, u, st in zip(wls, us, stats):
        assert st.status in (0, 4), (wl.name, st.status_name)
        uo, so = O.newton(O.build_problem(wl), tol=1e-14, max_iter=40)
        ug = host(u)
        assert relerr(ug, uo) < 1e-10, wl.name
        assert np.abs(ug - uo).max() <= 1e-10 * np.abs(uo).max(), wl.name


def test_batch_autotune_plan_solves_to_oracle(tmp_path):
    """The library's batch autotuner returns a plan kind, workgroup size and
    exponent from its candidates; the plan built with them solves every
    instance to the oracle's solution; the cached choice is returned without
    retiming."""
    E = eg()
    wls = [W.nonlinear_diffusion_2d(n, seed=200 + n) for n in (10, 21, 33)] + [W.nonlinear_diffusion_1d(40)]
    Ts, Ps = setup(wls)
    us = [torch.zeros(T.n, dtype=torch.float64, device=DEV) for T in Ts]
    opts = E.NewtonOptions(tol=1e-14, max_newton=40, krylov_rtol=1e-14)
    cache = str(tmp_path / "batch.json")
    res = E.batch_autotune(Ts, Ps, us, opts, cache=cache)
    if res["kind"] == 0:
        assert res["threads"] in (512, 1024) and res["weight_exp"] in (1.0, 1.5, 2.0)
    else:
        assert res["kind"] == 1 and res["threads"] in (256, 512) and res["weight_exp"] in (0.5, 1.0)
    assert res["ms"] > 0
    assert E.batch_autotune(Ts, Ps, us, opts, cache=cache) == res
    B = E.Batch(Ts, Ps, us, opts, threads=res["threads"], weight_exp=res["weight_exp"], kind=res["kind"])
    B.run(zero_init=True, graph=True)
    stats, rc = B.stats()
    B.close()
    assert rc in (0, 4)
    for wl, u, st in zip(wls, us, stats):
        assert st.status in (0, 4), st.status_name
        uo, _ = O.newton(O.build_problem(wl), tol=1e-14, max_iter=40)
        assert relerr(host(u), uo) < 1e-10, wl.name


SCHED_SIZES = (5, 17, 24, 40, 64)


def sched_mixed():
    return [W.nonlinear_diffusion_2d(n, seed=300 + n) for n in SCHED_SIZES] + \
        [W.nonlinear_diffusion_1d(64), W.semilinear_2d(20)]


@pytest.mark.parametrize("threads", [256, 512])
def test_sched_batch_matches_oracle(threads):
    """Scheduled resident teams (one row per thread, block-Jacobi BiCGStab on
    each member's rows): every instance solved tightly equals the oracle's
    Newton solution element-wise; the statistics name the resident
    block-Jacobi kernel; every team member holds at most `threads` rows."""
    E = eg()
    print(f"sched batch threads={threads}", flush=True)
    wls = sched_mixed()
    Ts, Ps = setup(wls)
    us = [torch.zeros(T.n, dtype=torch.float64, device=DEV) for T in Ts]
    opts = E.NewtonOptions(tol=1e-14, max_newton=40, krylov_rtol=1e-14)
    B = E.Batch(Ts, Ps, us, opts, threads=threads, kind=1)
    teams, total = B.teams()
    for T, g in zip(Ts, teams):
        assert g * threads >= T.n and g <= total
    B.run(zero_init=True)
    stats, rc = B.stats()
    B.close()
    assert rc in (0, 4), rc
    for wl, u, st in zip(wls, us, stats):
        assert st.status in (0, 4), (wl.name, st.status_name)
        assert st.krylov_kernels == 5
        uo, _ = O.newton(O.build_problem(wl), tol=1e-14, max_iter=40)
        ug = host(u)
        assert relerr(ug, uo) < 1e-10, wl.name
        assert np.abs(ug - uo).max() <= 1e-10 * np.abs(uo).max(), wl.name


def test_sched_batch_graph_replays_equal_eager():
    """A scheduled batch in which workgroups run several instances each:
    graph replays, with the program's eager work between them, equal the eager
    run bitwise (solutions and statistics)."""
    E = eg()
    wls = [W.nonlinear_diffusion_2d(n, seed=400 + n) for n in (12, 33, 48, 64, 100, 128)]
    Ts, Ps = setup(wls)
    us = [torch.full((T.n,), 0.3, dtype=torch.float64, device=DEV) for T in Ts]
    B = E.Batch(Ts, Ps, us, E.NewtonOptions(tol=1e-10, forcing=1), threads=256, kind=1)
    B.run(zero_init=True)
    st0, rc0 = B.stats()
    assert rc0 == 0
    eager = [host(u).copy() for u in us]
    for rep in range(3):
        for u in us:
            u.fill_(float(rep + 1))
        torch.cuda.synchronize()
        B.run(zero_init=True, graph=True)
        st, rc = B.stats()
        assert rc == 0
        for e, u, s, s0 in zip(eager, us, st, st0):
            assert np.array_equal(host(u), e), rep
            assert s.newton_iters == s0.newton_iters and s.krylov_iters == s0.krylov_iters
            assert s.res_hist == s0.res_hist
    B.close()


def test_sched_batch_rejections():
    """The scheduled teams take P1 handles with rows of at most 8 entries and
    workgroups of 256 or 512 threads."""
    E = eg()
    wls = [W.nonlinear_diffusion_2d(10, seed=5), W.diffusion_3d(4)]
    Ts, Ps = setup(wls)
    us = [torch.zeros(T.n, dtype=torch.float64, device=DEV) for T in Ts]
    with pytest.raises(E.EgfemError):
        E.Batch(Ts, Ps, us, kind=1)                     # 3D rows hold 15 entries
    with pytest.raises(E.EgfemError):
        E.Batch(Ts[:1], Ps[:1], us[:1], threads=1024, kind=1)
    with pytest.raises(E.EgfemError):
        E.Batch(Ts[:1], Ps[:1], us[:1], kind=2)
    B = E.Batch(Ts[:1], Ps[:1], us[:1], kind=1)
    B.run()
    stats, rc = B.stats()
    B.close()
    assert rc == 0 and stats[0].krylov_kernels == 5
