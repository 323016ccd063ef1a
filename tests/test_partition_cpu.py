"""Host logic of the block-Jacobi preconditioner: the compact row partition
(recursive coordinate bisection, one part per workgroup), run through the
library's own partition source built with g++ and checked here.

Checked: the parts cover every row exactly once, in ascending order within a
part, with balanced sizes; the part-local column positions are those of the
partition; the neighbour lists are exact, or all marked overflowed when any
part has more neighbour parts than a list holds; the part offsets and row
lists equal a brute-force bisection (split along the axis of largest extent,
nodes ordered by coordinate then id, the first half of the parts receiving
the proportional share of the nodes); invalid requests are rejected."""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIP_INCLUDE = "/opt/rocm/include"


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.isdir(HIP_INCLUDE):
        pytest.skip("g++ or the HIP headers are not available")
    exe = str(tmp_path_factory.mktemp("partition") / "partition_dump")
    subprocess.run(["g++", "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I" + HIP_INCLUDE,
                    os.path.join(ROOT, "tests", "partition_dump.cpp"),
                    os.path.join(ROOT, "paper_2005_06193_amd", "csrc", "egfem_partition.cpp"), "-o", exe],
                   check=True, capture_output=True)
    return exe


def wheel_mesh(k, seed=5):
    """A wheel with k rim nodes per ring: the centre node couples to every
    inner-ring node, so with many parts its part has many neighbour parts."""
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
    return coords, np.array(cells, dtype=np.int64)


def mesh_graph(name):
    if name == "wheel_150":
        coords, cells = wheel_mesh(150)
    else:
        m = {"1d_n300": lambda: W.mesh_1d(300), "2d_n24": lambda: W.mesh_2d(24),
             "3d_n7": lambda: W.mesh_3d(7), "disk_n20": lambda: W.mesh_disk(20)}[name]()
        coords, cells = np.asarray(m.coords, np.float64), np.asarray(m.cells, np.int64)
    coords = coords.reshape(len(coords), -1)
    n, nl = len(coords), cells.shape[1]
    r = np.concatenate([cells[:, a] for a in range(nl) for b in range(nl)])
    c = np.concatenate([cells[:, b] for a in range(nl) for b in range(nl)])
    A = sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(n, n))
    A.sum_duplicates()
    A.sort_indices()
    return coords, A.indptr.astype(np.int32), A.indices.astype(np.int32)


def run_partition(driver, tmp_path, coords, rowptr, col, G):
    p = str(tmp_path / f"g{G}")
    n, dim = coords.shape
    np.asarray([dim, n], np.int64).tofile(p + ".hdr")
    np.ascontiguousarray(coords, np.float64).tofile(p + ".x")
    rowptr.tofile(p + ".rp")
    col.tofile(p + ".col")
    out = subprocess.run([driver, p, str(G)], check=True, capture_output=True, text=True).stdout
    rc = int(out.split()[1])
    if rc != 0:
        return rc, None
    meta = np.fromfile(p + ".meta", np.int32)
    return 0, dict(kr=np.fromfile(p + ".kr", np.int32), rlist=np.fromfile(p + ".rlist", np.int32),
                   kloc=np.fromfile(p + ".kloc", np.int16), nbr=np.fromfile(p + ".nbr", np.int32),
                   maxrows=int(meta[0]), lists=int(meta[1]))


def bisection(X, ids, parts):
    """Brute-force recursive coordinate bisection: the parts as lists of ids."""
    if parts == 1:
        return [sorted(ids)]
    sub = X[ids]
    ax = int(np.argmax(sub.max(0) - sub.min(0)))          # first axis of largest extent
    order = sorted(ids, key=lambda a: (X[a, ax], a))
    h = parts // 2
    cut = len(ids) * h // parts
    return bisection(X, order[:cut], h) + bisection(X, order[cut:], parts - h)


CASES = [("1d_n300", 1), ("1d_n300", 7), ("1d_n300", 300), ("2d_n24", 5), ("2d_n24", 64), ("3d_n7", 9),
         ("3d_n7", 40), ("disk_n20", 13), ("wheel_150", 4), ("wheel_150", 64)]


@pytest.mark.parametrize("name,G", CASES, ids=[f"{m}-G{g}" for m, g in CASES])
def test_compact_partition(driver, tmp_path, name, G):
    coords, rowptr, col = mesh_graph(name)
    n = len(coords)
    rc, P = run_partition(driver, tmp_path, coords, rowptr, col, G)
    assert rc == 0
    kr, rlist, kloc, L = P["kr"], P["rlist"], P["kloc"], P["lists"]
    # cover, order, balance
    assert len(kr) == G + 1 and kr[0] == 0 and kr[G] == n
    sizes = np.diff(kr)
    assert sizes.min() >= n // G and sizes.max() <= -(-n // G)
    assert P["maxrows"] == sizes.max()
    assert np.array_equal(np.sort(rlist), np.arange(n))
    owner = np.empty(n, np.int64)
    pos = np.empty(n, np.int64)
    for g in range(G):
        rows = rlist[kr[g]:kr[g + 1]]
        assert np.all(np.diff(rows) > 0)
        owner[rows] = g
        pos[rows] = np.arange(len(rows))
    # part-local column positions
    row_of = np.repeat(np.arange(n), np.diff(rowptr))
    same = owner[col] == owner[row_of]
    assert np.array_equal(kloc, np.where(same, pos[col], -1).astype(np.int16))
    # neighbour lists: exact, or all overflowed
    nbr = P["nbr"].reshape(G, L + 1)
    want = [sorted(set(owner[col[owner[row_of] == g]].tolist()) - {g}) for g in range(G)]
    if max(len(w) for w in want) > L:
        assert np.all(nbr[:, 0] == -1)
    else:
        for g in range(G):
            assert nbr[g, 0] == len(want[g])
            assert sorted(nbr[g, 1:1 + nbr[g, 0]].tolist()) == want[g]
    # the bisection itself
    parts = bisection(coords, list(range(n)), G)
    assert np.array_equal(kr, np.cumsum([0] + [len(q) for q in parts]))
    assert np.array_equal(rlist, np.concatenate([np.asarray(q, np.int32) for q in parts]))


def test_wheel_many_parts_overflow_every_list(driver, tmp_path):
    """64 parts of a wheel with 150 nodes per ring: the centre node's part sees
    more neighbour parts than a list holds, so every list is marked overflowed
    (all workgroups then take the team barrier)."""
    coords, rowptr, col = mesh_graph("wheel_150")
    rc, P = run_partition(driver, tmp_path, coords, rowptr, col, 64)
    assert rc == 0
    assert np.all(P["nbr"].reshape(64, P["lists"] + 1)[:, 0] == -1)


@pytest.mark.parametrize("G", [0, -3, 302])
def test_invalid_part_count_rejected(driver, tmp_path, G):
    coords, rowptr, col = mesh_graph("1d_n300")           # 301 nodes
    rc, P = run_partition(driver, tmp_path, coords, rowptr, col, G)
    assert rc != 0 and P is None


# Host model of the indexing of the register-resident Krylov kernels with the
# block-Jacobi preconditioner (one thread per row of the workgroup's part,
# rows of at most K = 8 entries, LDS step buffers of 2 vectors x (NT + 1)
# doubles, entry NT of each an always-zero value).  Checked for every
# workgroup and every thread, also where a part is far smaller than the
# workgroup: the clamped row of a thread without a row, the clamped entry
# index, the part-local position of an in-block column (it must name that
# column's row in the same part), and every LDS index read or written.
K_RESIDENT = 8
MODEL_CASES = [("1d_n300", 2, 256), ("1d_n300", 2, 512), ("1d_n300", 5, 256), ("1d_n300", 300, 256),
               ("2d_n24", 5, 256), ("2d_n24", 3, 512), ("2d_n24", 64, 256), ("disk_n20", 13, 256)]


@pytest.mark.parametrize("name,G,NT", MODEL_CASES, ids=[f"{m}-G{g}-NT{t}" for m, g, t in MODEL_CASES])
def test_resident_block_jacobi_indexing_model(driver, tmp_path, name, G, NT):
    coords, rowptr, col = mesh_graph(name)
    n, S = len(coords), len(col)
    rc, P = run_partition(driver, tmp_path, coords, rowptr, col, G)
    assert rc == 0
    kr, rlist, kloc = P["kr"], P["rlist"], P["kloc"]
    assert P["maxrows"] <= NT                       # the launcher's condition for the resident form
    assert np.diff(rowptr).max() <= K_RESIDENT
    lds_words = 4 * (NT + 1)                         # two buffers x two vectors
    for g in range(G):
        rb, re = int(kr[g]), int(kr[g + 1])
        written = set()
        for tid in range(NT):
            i = rb + tid
            own = i < re
            q = max(min(i, re - 1), 0)
            assert 0 <= q < n
            row = int(rlist[q])
            beg, end = int(rowptr[row]), int(rowptr[row + 1])
            for k in range(K_RESIDENT):
                vi = min(beg + k, end - 1)
                assert 0 <= vi < S
                c = int(col[vi])
                offd = own and beg + k < end and c != row
                l = int(kloc[vi])
                li = l if (offd and l >= 0) else NT
                assert 0 <= li <= NT
                if li < NT:
                    assert li < re - rb and int(rlist[rb + li]) == c   # the column's own row in the part
                for v in range(2):
                    for buf in range(2):
                        assert buf * 2 * (NT + 1) + v * (NT + 1) + li < lds_words
            for v in range(2):
                for buf in range(2):
                    idx = buf * 2 * (NT + 1) + v * (NT + 1) + tid
                    assert idx < lds_words
                    written.add(idx)
        # the zero entries (index NT of each vector and buffer) are written by
        # threads 0..3 and by no row thread
        zeros = {(t >> 1) * 2 * (NT + 1) + (t & 1) * (NT + 1) + NT for t in range(4)}
        assert len(zeros) == 4 and not (zeros & written)
