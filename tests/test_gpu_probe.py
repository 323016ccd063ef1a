"""Measurement aids on the GPU: the streaming-read ceiling probe
(egfem_stream_read) sums every chunk like a plain reduction, and the raw
tensor action replayed from a captured graph equals the eager launch."""
import numpy as np
import pytest
import torch

import workloads as W
from paper_2005_06193_amd import binding as B
from test_gpu_parity import DEV, eg

pytestmark = pytest.mark.gpu

CHUNK = 2048


@pytest.mark.parametrize("n", [1, 2047, 2048, 2049, 3 * 2048 + 5, 1 << 20])
@pytest.mark.parametrize("offset", [0, 1])
def test_stream_read_chunk_sums(n, offset):
    """partial[c] is the sum of chunk c (full chunks on the 16-byte vector
    path when aligned, the scalar path otherwise and for the short tail)."""
    E = eg()
    print(f"stream_read n={n} offset={offset}", flush=True)
    base = torch.rand(n + offset, dtype=torch.float64, device=DEV)
    x = base[offset:]
    assert E.load_library().egfem_stream_read_chunks(n) == (n + CHUNK - 1) // CHUNK
    part = E.stream_read(x)
    torch.cuda.synchronize()
    h = x.cpu().numpy()
    nc = (n + CHUNK - 1) // CHUNK
    want = np.array([h[c * CHUNK:(c + 1) * CHUNK].sum() for c in range(nc)])
    got = part.cpu().numpy()[:nc]
    assert np.allclose(got, want, rtol=1e-13, atol=0.0)


def test_stream_read_edges():
    E = eg()
    lib = E.load_library()
    assert lib.egfem_stream_read_chunks(0) == 0
    x = torch.ones(4096, dtype=torch.float64, device=DEV)
    short = torch.empty(1, dtype=torch.float64, device=DEV)
    with pytest.raises(E.EgfemError):
        E.stream_read(x, short)                  # two chunks, one partial
    assert lib.egfem_stream_read(None, 0, None, 0, None) == 0
    assert lib.egfem_stream_read(None, 5, None, 1, None) == B.EGFEM_ERR_ARG


def test_action_graph_replays_equal_eager():
    """20 raw actions captured in one graph, replayed three times with eager
    work and synchronisations between the replays: every replay's result is
    bitwise the eager action's."""
    E = eg()
    wl = W.nonlinear_diffusion_2d(48)
    T = E.Tensor.from_mesh(wl.mesh, wl.form)
    g = torch.Generator(device=DEV).manual_seed(9)
    u = torch.rand(T.n, dtype=torch.float64, device=DEV, generator=g)
    a = torch.rand(T.n, dtype=torch.float64, device=DEV, generator=g) + 1.0
    r = torch.empty_like(u)
    ref = torch.empty_like(u)
    T.residual(u, a, ref)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        T.residual(u, a, r)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(20):
            T.residual(u, a, r)
    for rep in range(3):
        r.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(r, ref), rep
        T.residual(a, u, ref)                    # eager work between replays
        T.residual(u, a, ref)
        torch.cuda.synchronize()
    del graph
    T.close()
