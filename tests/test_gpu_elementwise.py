"""Storage variants against the oracle's tensor contraction and against the
slot-aligned stream action of the same handle: the element-factored form of
the stiffness tensor (T^e = K^e / (d+1) on every cell), and the unique storage
of the fully symmetric mass tensor (one value per index multiset)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import egfem_oracle as O
from test_gpu_parity import DEV, dt, eg, host, irregular_mesh, relerr

pytestmark = pytest.mark.gpu

MESHES = {
    "1d_n33": lambda: W.mesh_1d(33),
    "2d_n8": lambda: W.mesh_2d(8),
    "2d_n45": lambda: W.mesh_2d(45),
    "2d_jitter_n21": lambda: irregular_mesh(21),
    "3d_n3": lambda: W.mesh_3d(3),
    "3d_n9": lambda: W.mesh_3d(9),
}


@pytest.mark.parametrize("mesh", list(MESHES))
def test_elementwise_action_matches_oracle_and_stream(mesh):
    m = MESHES[mesh]()
    print(f"elementwise {mesh}", flush=True)
    T = eg().Tensor.from_mesh(m, W.FORM_STIFF)
    T.attach_elements(m.coords, m.cells)
    To = O.assemble_tensor(m.coords, m.cells, O.FORM_STIFF)
    rng = np.random.default_rng(29)
    u = rng.uniform(-1, 1, m.n_nodes)
    a = rng.uniform(0.5, 2, m.n_nodes)
    re = host(T.residual_elementwise(dt(u), dt(a)))
    assert relerr(re, O.contract_uv(To, u, a)) < 1e-12
    rs = host(T.residual(dt(u), dt(a)))
    assert np.abs(re - rs).max() <= 1e-13 * np.abs(rs).max()
    # a constant u lies in the kernel of every K^e
    z = host(T.residual_elementwise(dt(np.full(m.n_nodes, 3.0)), dt(a)))
    assert np.abs(z).max() <= 1e-13 * np.abs(rs).max()


def test_elementwise_full_size_and_errors():
    m = W.mesh_2d(256)
    T = eg().Tensor.from_mesh(m, W.FORM_STIFF)
    x = dt(np.ones(T.n))
    with pytest.raises(eg().EgfemError):
        T.residual_elementwise(x, x)                   # nothing attached yet
    T.attach_elements(m.coords, m.cells)
    rng = np.random.default_rng(31)
    u = rng.uniform(-1, 1, T.n)
    a = rng.uniform(0.5, 2, T.n)
    re = host(T.residual_elementwise(dt(u), dt(a)))
    rs = host(T.residual(dt(u), dt(a)))
    assert np.abs(re - rs).max() <= 1e-13 * np.abs(rs).max()
    # re-attaching replaces the data and gives the same result
    T.attach_elements(m.coords, m.cells)
    assert np.array_equal(host(T.residual_elementwise(dt(u), dt(a))), re)
    # wrong form, wrong mesh
    M = eg().Tensor.from_mesh(W.mesh_2d(8), W.FORM_MASS)
    with pytest.raises(eg().EgfemError):
        M.attach_elements(W.mesh_2d(8).coords, W.mesh_2d(8).cells)
    with pytest.raises(eg().EgfemError):
        T.attach_elements(W.mesh_2d(8).coords, W.mesh_2d(8).cells)


# ----------------------------------------------------------------------------
# unique storage of the fully symmetric mass tensor (one value per multiset)
# ----------------------------------------------------------------------------
def _multiset_count(m):
    import itertools
    edges, faces = set(), set()
    for c in m.cells:
        c = sorted(int(x) for x in c)
        edges.update(itertools.combinations(c, 2))
        faces.update(itertools.combinations(c, 3))
    return m.n_nodes + 2 * len(edges) + len(faces)


def _abs_tensor(T):
    return O.Tensor3(T.n, T.i, T.j, T.k, np.abs(T.v))


@pytest.mark.parametrize("mesh", list(MESHES))
def test_unique_mass_action_matches_oracle_and_stream(mesh):
    m = MESHES[mesh]()
    print(f"unique mass {mesh}", flush=True)
    T = eg().Tensor.from_mesh(m, W.FORM_MASS)
    nu = T.attach_unique(m.coords, m.cells)
    assert nu == _multiset_count(m)
    To = O.assemble_tensor(m.coords, m.cells, O.FORM_MASS)
    rng = np.random.default_rng(37)
    u = rng.uniform(-1, 1, m.n_nodes)
    a = rng.uniform(-2, 2, m.n_nodes)
    ru = host(T.residual_unique(dt(u), dt(a)))
    ro = O.contract_uv(To, u, a)
    # each term within a few ulps of the sum of |terms|
    scale = O.contract_uv(_abs_tensor(To), np.abs(u), np.abs(a))
    assert np.all(np.abs(ru - ro) <= 1e-14 * scale)
    rs = host(T.residual(dt(u), dt(a)))
    assert np.all(np.abs(ru - rs) <= 1e-14 * scale)
    # T:(1 (x) a) = M a (mass matrix times a); u = a gives the symmetric form
    ones = host(T.residual_unique(dt(np.ones(m.n_nodes)), dt(a)))
    Ma = O.assemble_mass(m.coords, m.cells) @ a
    assert np.abs(ones - Ma).max() <= 1e-14 * np.abs(O.assemble_mass(m.coords, m.cells)).sum(axis=1).max() * 2
    # deterministic
    assert np.array_equal(host(T.residual_unique(dt(u), dt(a))), ru)


def test_unique_mass_full_size_2d_512_and_errors():
    """2D 512x512 (the mass workload of the action measurements): sampled rows
    against the oracle's row assembly, every row against the stream."""
    m = W.mesh_2d(512)
    print("unique mass 2d_512 full size", flush=True)
    T = eg().Tensor.from_mesh(m, W.FORM_MASS)
    x = dt(np.ones(T.n))
    with pytest.raises(eg().EgfemError):
        T.residual_unique(x, x)                        # nothing attached yet
    nu = T.attach_unique(m.coords, m.cells)
    assert nu == 9 * 512 * 512 + 6 * 512 + 1
    rng = np.random.default_rng(41)
    u = rng.uniform(-1, 1, T.n)
    a = rng.uniform(0.5, 2, T.n)
    ru = host(T.residual_unique(dt(u), dt(a)))
    rs = host(T.residual(dt(u), dt(a)))
    assert np.abs(ru - rs).max() <= 1e-14 * np.abs(rs).max()
    rows = np.unique(np.concatenate([np.arange(0, 40), rng.integers(0, T.n, 200), np.arange(T.n - 40, T.n)]))
    Tr = O.tensor_rows(m.coords, m.cells, O.FORM_MASS, rows)
    ro = O.contract_uv(Tr, u, a)[rows]
    assert np.abs(ru[rows] - ro).max() <= 1e-14 * np.abs(ro).max()
    # re-attaching replaces the data and gives the same result
    T.attach_unique(m.coords, m.cells)
    assert np.array_equal(host(T.residual_unique(dt(u), dt(a))), ru)
    # wrong form, wrong coefficient space, wrong mesh
    small = W.mesh_2d(8)
    S = eg().Tensor.from_mesh(small, W.FORM_STIFF)
    with pytest.raises(eg().EgfemError):
        S.attach_unique(small.coords, small.cells)
    P = eg().Tensor.from_mesh(small, W.FORM_MASS, wspace=eg().W_P2)
    with pytest.raises(eg().EgfemError):
        P.attach_unique(small.coords, small.cells)
    with pytest.raises(eg().EgfemError):
        T.attach_unique(small.coords, small.cells)
    # same sizes, other cells (a different diagonal in one square): pattern mismatch
    M8 = eg().Tensor.from_mesh(small, W.FORM_MASS)
    cells = small.cells.copy()
    q0, q1 = cells[0].copy(), cells[1].copy()
    quad = sorted(set(q0.tolist()) | set(q1.tolist()))
    if len(quad) == 4:
        shared = sorted(set(q0.tolist()) & set(q1.tolist()))
        other = [v for v in quad if v not in shared]
        cells[0] = [other[0], other[1], shared[0]]
        cells[1] = [other[0], other[1], shared[1]]
        with pytest.raises(eg().EgfemError):
            M8.attach_unique(small.coords, cells)
