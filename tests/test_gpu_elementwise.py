"""Element-factored form of the stiffness tensor (T^e = K^e / (d+1) on every
cell): its action against the oracle's tensor contraction and against the
slot-aligned stream action of the same handle."""
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
