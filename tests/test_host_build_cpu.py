"""The library's offline tensor build as host code under the address and
undefined-behaviour sanitizers (g++, no GPU): its build source is linked
against a host-memory stand-in for the HIP allocation and copy calls
(tests/host_build_dump.cpp), run on small 1D, 2D, jittered 2D and 3D meshes
for every form and coefficient space, and the stored tensor is compared entry
by entry with the oracle's (same (i, j, k) set, values to 1e-14 of the row's
largest entry).  The block-relative stream format is checked against the
global streams inside the driver.  Any sanitizer report fails the run."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as W
from oracle import egfem_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIP_INCLUDE = "/opt/rocm/include"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.isdir(HIP_INCLUDE):
        pytest.skip("g++ or the HIP headers are not available")
    exe = str(tmp_path_factory.mktemp("hostbuild") / "host_build_dump")
    r = subprocess.run(["g++", "-O1", "-g", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I" + HIP_INCLUDE,
                        "-I" + os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "host_build_dump.cpp"),
                        os.path.join(ROOT, "paper_2005_06193_amd", "csrc", "egfem_build.cpp"), "-o", exe],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail("g++ build of the host driver failed:\n" + r.stderr[-4000:])
    return exe


def jittered_2d(n, seed=11):
    m = W.mesh_2d(n)
    rng = np.random.default_rng(seed)
    x = np.array(m.coords, dtype=np.float64)
    inner = ~np.asarray(m.dirichlet, bool)
    x[inner] += rng.uniform(-0.2, 0.2, (int(inner.sum()), 2)) / n
    return x, np.asarray(m.cells)


MESHES = {
    "1d_9": lambda: (W.mesh_1d(9).coords, W.mesh_1d(9).cells),
    "2d_6": lambda: (W.mesh_2d(6).coords, W.mesh_2d(6).cells),
    "2d_jitter_7": lambda: jittered_2d(7),
    "3d_3": lambda: (W.mesh_3d(3).coords, W.mesh_3d(3).cells),
}


def run_build(driver, tmp_path, coords, cells, form, wspace=0):
    coords = np.asarray(coords, np.float64).reshape(len(coords), -1)
    cells = np.asarray(cells, np.int32)
    n, dim = coords.shape
    p = str(tmp_path / f"m{form}{wspace}")
    np.asarray([dim, n, len(cells), form, wspace], np.int64).tofile(p + ".hdr")
    coords.tofile(p + ".x")
    cells.tofile(p + ".cells")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([driver, p], capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    kv = {}
    for line in r.stdout.split("\n"):
        parts = line.split()
        for a, b in zip(parts[0::2], parts[1::2]):
            kv[a] = int(b)
    return p, kv, r.stdout


@pytest.mark.parametrize("mesh", sorted(MESHES))
@pytest.mark.parametrize("form", [O.FORM_STIFF, O.FORM_MASS, O.FORM_CONV])
def test_host_build_matches_oracle_under_sanitizers(driver, tmp_path, mesh, form):
    coords, cells = MESHES[mesh]()
    p, kv, out = run_build(driver, tmp_path, coords, cells, form)
    assert kv["rc"] == 0, out
    assert kv["block_mismatch"] == 0, out
    if form == O.FORM_MASS:
        assert "unique_rc 0" in out, out
    if form == O.FORM_STIFF:
        assert "elements_rc 0" in out, out
    I, J, K = (np.fromfile(p + s, np.int32) for s in (".i", ".j", ".k"))
    V = np.fromfile(p + ".v", np.float64)
    ref = O.assemble_tensor(np.asarray(coords, np.float64).reshape(len(coords), -1), np.asarray(cells), form)
    n = ref.n
    key = (I.astype(np.int64) * n + J) * n + K
    rkey = (ref.i.astype(np.int64) * n + ref.j) * n + ref.k
    o, ro = np.argsort(key), np.argsort(rkey)
    assert np.array_equal(key[o], rkey[ro])
    rowmax = np.zeros(n)
    np.maximum.at(rowmax, ref.i, np.abs(ref.v))
    assert np.all(np.abs(V[o] - ref.v[ro]) <= 1e-14 * rowmax[ref.i[ro]])
    assert kv["nnz"] == ref.nnz


@pytest.mark.parametrize("mesh", sorted(MESHES))
@pytest.mark.parametrize("wspace", [1, 2, 3])
def test_host_build_coefficient_spaces_under_sanitizers(driver, tmp_path, mesh, wspace):
    """W_h = P2, I_k and P0 handles (stiffness and mass forms; P2 and I_k also
    the convection form) build without a sanitizer report; the stored entry
    count equals the oracle's tensor on that space, and the B position of
    every entry names the same entry in the W-slot-aligned B stream."""
    coords, cells = MESHES[mesh]()
    coords = np.asarray(coords, np.float64).reshape(len(coords), -1)
    cells = np.asarray(cells)
    forms = [O.FORM_STIFF, O.FORM_MASS] + ([O.FORM_CONV] if wspace in (1, 2) else [])
    for form in forms:
        if wspace == 3 and form == O.FORM_MASS:
            continue
        _, kv, out = run_build(driver, tmp_path, coords, cells, form, wspace)
        assert kv["rc"] == 0, out
        assert kv["block_mismatch"] == 0, (form, out)
        if wspace == 1:
            ref = O.tensor_p2(coords, cells, form)
        elif wspace == 2:
            ref = O.tensor_iq(coords, cells, form)
        else:
            ref = O.tensor_p0(coords, cells)
        ref = ref[0] if isinstance(ref, tuple) else ref
        assert kv["nnz"] == ref.nnz, (form, out)
