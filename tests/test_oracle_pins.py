"""Pins of the CPU oracle against facts fixed by the mathematics or printed in
the paper (not against the oracle itself).  CPU only."""
import math
import itertools
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import egfem_oracle as O


# ----------------------------------------------------------------------------
# exact rational helpers (brute force, independent of the oracle's numpy code)
# ----------------------------------------------------------------------------
def _frac_inv(B):
    n = len(B)
    A = [[Fraction(B[r][c]) for c in range(n)] + [Fraction(int(r == c)) for c in range(n)]
         for r in range(n)]
    for c in range(n):
        p = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[p] = A[p], A[c]
        piv = A[c][c]
        A[c] = [x / piv for x in A[c]]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c]
                A[r] = [x - f * y for x, y in zip(A[r], A[c])]
    return [row[n:] for row in A]


def _frac_det(B):
    n = len(B)
    if n == 1:
        return Fraction(B[0][0])
    return sum((-1) ** c * Fraction(B[0][c]) *
               _frac_det([row[:c] + row[c + 1:] for row in B[1:]]) for c in range(n))


def _exact_element(verts):
    """grad lambda_a (exact rationals) and |e| for one simplex."""
    d = len(verts) - 1
    x0 = verts[0]
    B = [[Fraction(verts[m + 1][r]) - Fraction(x0[r]) for m in range(d)] for r in range(d)]
    Binv = _frac_inv(B)
    vol = abs(_frac_det(B)) / math.factorial(d)
    grads = [[-sum(Binv[m][r] for m in range(d)) for r in range(d)]] + [Binv[m] for m in range(d)]
    return grads, vol


def _int_monomial(alpha, vol, d):
    """int_e prod lambda_a^alpha_a = d! prod(alpha_a!) |e| / (d + |alpha|)!"""
    return Fraction(math.factorial(d) * math.prod(math.factorial(a) for a in alpha),
                    math.factorial(d + sum(alpha))) * vol


def _exact_tensor(coords, cells, form):
    n, d = coords.shape
    T = {}
    for cell in cells:
        verts = [[Fraction(float(x)) for x in coords[v]] for v in cell]
        grads, vol = _exact_element(verts)
        for a, b, c in itertools.product(range(d + 1), repeat=3):
            if form == O.FORM_STIFF:
                gg = sum(grads[a][r] * grads[b][r] for r in range(d))
                al = [0] * (d + 1)
                al[c] += 1
                val = gg * _int_monomial(al, vol, d)
            elif form == O.FORM_CONV:
                al = [0] * (d + 1)
                al[b] += 1
                al[c] += 1
                val = sum(grads[a][r] for r in range(d)) * _int_monomial(al, vol, d)
            else:
                al = [0] * (d + 1)
                for x in (a, b, c):
                    al[x] += 1
                val = _int_monomial(al, vol, d)
            key = (int(cell[a]), int(cell[b]), int(cell[c]))
            T[key] = T.get(key, Fraction(0)) + val
    return {k: v for k, v in T.items() if v != 0}


def _as_dict(T: O.Tensor3):
    return {(int(i), int(j), int(k)): float(v) for i, j, k, v in zip(T.i, T.j, T.k, T.v)}


IRREGULAR = {
    1: (np.array([[0.0], [0.375], [1.0]]), np.array([[0, 1], [1, 2]], dtype=np.int32)),
    2: (np.array([[0.0, 0.0], [0.75, 0.125], [0.25, 0.625], [1.0, 0.875]]),
        np.array([[0, 1, 2], [1, 3, 2]], dtype=np.int32)),
    3: (np.array([[0.0, 0.0, 0.0], [0.75, 0.125, 0.0], [0.25, 0.625, 0.125],
                  [0.125, 0.25, 0.5], [0.875, 0.75, 0.625]]),
        np.array([[0, 1, 2, 3], [1, 2, 3, 4]], dtype=np.int32)),
}


# ----------------------------------------------------------------------------
# quadrature
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [1, 2, 3])
def test_quadrature_exact_for_monomials(dim):
    for deg in range(0, 7):
        X, Wt = O.simplex_quadrature(dim, deg)
        lam = O.barycentric(X)
        assert abs(Wt.sum() - 1.0 / math.factorial(dim)) < 1e-15
        for alpha in itertools.product(range(deg + 1), repeat=dim + 1):
            if sum(alpha) > deg:
                continue
            num = np.sum(Wt * np.prod(lam ** np.array(alpha), axis=1))
            ex = float(_int_monomial(alpha, Fraction(1, math.factorial(dim)), dim))
            assert abs(num - ex) < 1e-15


# ----------------------------------------------------------------------------
# meshes and the sizes printed in the paper
# ----------------------------------------------------------------------------
def test_mesh_counts_and_volume():
    for dim, n, nodes, cells in [(1, 256, 257, 256), (2, 256, 66049, 131072),
                                 (2, 512, 263169, 524288), (3, 16, 17 ** 3, 6 * 16 ** 3)]:
        m = W.structured_mesh(dim, n)
        assert m.n_nodes == nodes and m.n_cells == cells
        det, _ = O.element_geometry(m.coords, m.cells)
        assert abs(det.sum() / math.factorial(dim) - 1.0) < 1e-12


def test_table1_system_sizes():
    """Sizes of Table tbl:superconductivity (Sec. 5.3) on the 64x64 triangle mesh."""
    rows = {}
    with open(__file__.replace("test_oracle_pins.py", "golden/table1_sizes.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                name, size = line.split()
                rows[name] = int(size)
    m = W.mesh_2d(64)
    p2 = O.p2_space(m.coords, m.cells)
    n_u, n_el = m.n_nodes, m.n_cells
    n_edges = p2.edges.shape[0]
    assert rows["SGA"] == n_u                              # u only
    assert rows["GFEM"] == 2 * n_u                         # u + c on V_h
    assert rows["EGFEM_P2"] == n_u + p2.n_w                # u + c on P2
    assert rows["EGFEM_P3"] == n_u + n_u + 2 * n_edges + n_el   # P3: vertices, 2/edge, 1/cell
    assert rows["EGFEM_I4"] == n_u + 6 * n_el              # 6-point degree-4 rule per triangle


# ----------------------------------------------------------------------------
# matrices
# ----------------------------------------------------------------------------
def test_stiffness_is_finite_difference_stencil():
    n = 8
    h = 1.0 / n
    K1 = O.assemble_stiffness(*(lambda m: (m.coords, m.cells))(W.mesh_1d(n))).toarray()
    assert np.allclose(K1[3, 2:5], [-1 / h, 2 / h, -1 / h], atol=1e-12)
    m = W.mesh_2d(n)
    K2 = O.assemble_stiffness(m.coords, m.cells).toarray()
    i = 3 * (n + 1) + 4
    row = K2[i]
    assert abs(row[i] - 4.0) < 1e-13
    for o in (1, -1, n + 1, -(n + 1)):
        assert abs(row[i + o] + 1.0) < 1e-13
    assert np.sum(np.abs(row) > 1e-13) == 5
    m = W.mesh_3d(4)
    K3 = O.assemble_stiffness(m.coords, m.cells).toarray()
    s = 5
    i = (2 * s + 2) * s + 2
    row = K3[i]
    h = 0.25
    assert abs(row[i] - 6 * h) < 1e-13
    for o in (1, -1, s, -s, s * s, -s * s):
        assert abs(row[i + o] + h) < 1e-13
    assert np.sum(np.abs(row) > 1e-13) == 7


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_mass_matrix(dim):
    m = W.structured_mesh(dim, 4)
    M = O.assemble_mass(m.coords, m.cells)
    assert abs(M.sum() - 1.0) < 1e-13
    # consistent mass: M_aa = 2|e|/((d+1)(d+2)), M_ab = |e|/((d+1)(d+2)) per element
    coords, cells = IRREGULAR[dim]
    Mi = O.assemble_mass(coords, cells).toarray()
    ex = np.zeros_like(Mi)
    for cell in cells:
        _, vol = _exact_element([[Fraction(float(x)) for x in coords[v]] for v in cell])
        for a in cell:
            for b in cell:
                ex[a, b] += float(vol * (2 if a == b else 1) / ((dim + 1) * (dim + 2)))
    assert np.abs(Mi - ex).max() < 1e-15


# ----------------------------------------------------------------------------
# third-order tensors
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("form", [O.FORM_STIFF, O.FORM_MASS, O.FORM_CONV])
def test_tensor_matches_exact_rational_integrals(dim, form):
    coords, cells = IRREGULAR[dim]
    T = _as_dict(O.assemble_tensor(coords, cells, form, drop_rel=0.0))
    ex = _exact_tensor(coords, cells, form)
    assert set(T) == set(ex)
    scale = max(abs(float(v)) for v in ex.values())
    for key, v in ex.items():
        assert abs(T[key] - float(v)) <= 1e-14 * scale


def test_stiffness_tensor_identities():
    for dim, n in [(1, 8), (2, 6), (3, 3)]:
        m = W.structured_mesh(dim, n)
        T = O.assemble_tensor(m.coords, m.cells, O.FORM_STIFF)
        K = O.assemble_stiffness(m.coords, m.cells)
        # T . 1 = K  (sum over k of int psi_k grad.grad, partition of unity of psi)
        assert abs(O.contract_first(T, np.ones(T.n)) - K).max() < 1e-13
        D = T.dense()
        assert np.abs(D - D.transpose(1, 0, 2)).max() < 1e-14      # T_ijk = T_jik
        assert np.abs(D.sum(axis=1)).max() < 1e-13                   # sum_j grad phi_j = 0
        # per element T^e_ijk = K^e_ij / (d+1): with psi = 1 summed, equals K
        assert np.abs(D.sum(axis=2) - K.toarray()).max() < 1e-13


def test_mass_tensor_identities():
    for dim, n in [(1, 8), (2, 5), (3, 2)]:
        m = W.structured_mesh(dim, n)
        T = O.assemble_tensor(m.coords, m.cells, O.FORM_MASS)
        M = O.assemble_mass(m.coords, m.cells).toarray()
        D = T.dense()
        for perm in itertools.permutations(range(3)):
            assert np.abs(D - D.transpose(perm)).max() < 1e-16
        assert np.abs(D.sum(axis=2) - M).max() < 1e-15


def test_mass_tensor_unique_multisets():
    """The fully symmetric mass tensor holds one value per index multiset: N of
    the form iii, two per edge (iij, ijj), one per face (ijk), each stored in
    the full tensor once per distinct ordering (1, 3 or 6 entries); on the 2D
    n x n mesh N + 2E + F = 9 n^2 + 6 n + 1."""
    for dim, n in [(1, 7), (2, 4), (2, 7), (3, 2)]:
        m = W.structured_mesh(dim, n)
        T = O.assemble_tensor(m.coords, m.cells, O.FORM_MASS)
        groups = {}
        for i, j, k, v in zip(T.i, T.j, T.k, T.v):
            groups.setdefault(tuple(sorted((int(i), int(j), int(k)))), []).append(v)
        edges, faces = set(), set()
        for c in m.cells:
            c = sorted(int(x) for x in c)
            edges.update(itertools.combinations(c, 2))
            faces.update(itertools.combinations(c, 3))
        assert len(groups) == m.n_nodes + 2 * len(edges) + len(faces)
        for key, vals in groups.items():
            assert len(vals) == len(set(itertools.permutations(key)))
            assert max(vals) - min(vals) <= 1e-15 * max(vals)   # orderings summed in other orders
        assert T.nnz == m.n_nodes + 6 * len(edges) + 6 * len(faces)
        if dim == 2:
            assert len(groups) == 9 * n * n + 6 * n + 1


def test_tensor_nnz_closed_forms():
    for n in (2, 3, 5, 8, 12):
        m = W.mesh_2d(n)
        T = O.assemble_tensor(m.coords, m.cells, O.FORM_STIFF)
        assert T.nnz == 23 * n * n + 14 * n + 1
        assert T.structural_nnz == 31 * n * n + 14 * n + 1
        assert O.slot_count(T) == 5 * n * n + 6 * n + 1
        TM = O.assemble_tensor(m.coords, m.cells, O.FORM_MASS)
        assert TM.nnz == 31 * n * n + 14 * n + 1
        assert O.slot_count(TM) == 7 * n * n + 6 * n + 1
    for n in (2, 3, 4):
        m = W.mesh_3d(n)
        T = O.assemble_tensor(m.coords, m.cells, O.FORM_STIFF)
        assert T.nnz == 63 * n ** 3 + 69 * n ** 2 + 21 * n + 1
        assert T.structural_nnz == 115 * n ** 3 + 93 * n ** 2 + 21 * n + 1


# ----------------------------------------------------------------------------
# residual and Jacobian
# ----------------------------------------------------------------------------
def _small_problem(dim, n, form=O.FORM_STIFF, seed=5):
    rng = np.random.default_rng(seed)
    m = W.structured_mesh(dim, n)
    if form == O.FORM_STIFF:
        wl = W.Workload("t", m, rng.uniform(0, 10, m.n_nodes), form,
                        rng.uniform(0.5, 2.0, m.n_nodes) if dim == 3 else None, 1.0, False, 1e-12, seed)
    else:
        wl = W.Workload("t", m, rng.uniform(-50, 50, m.n_nodes), form, None, 0.0, True, 1e-12, seed)
    return O.build_problem(wl)


def test_residual_special_cases():
    p = _small_problem(2, 6)
    rng = np.random.default_rng(1)
    u = rng.uniform(-1, 1, p.n)
    K = O.assemble_stiffness(p.coords, p.cells)
    # constant a: T:(u (x) c 1) = c K u
    assert np.abs(O.contract_uv(p.T, u, np.full(p.n, 2.5)) - 2.5 * (K @ u)).max() < 1e-12
    # constant u: T:(c 1 (x) a) = 0 (sum_j grad phi_j = 0)
    assert np.abs(O.contract_uv(p.T, np.full(p.n, 1.7), rng.uniform(1, 2, p.n))).max() < 1e-12


@pytest.mark.parametrize("dim,n,form", [(1, 9, O.FORM_STIFF), (2, 5, O.FORM_STIFF),
                                        (3, 2, O.FORM_STIFF), (2, 5, O.FORM_MASS)])
def test_jacobian_taylor_and_fd(dim, n, form):
    p = _small_problem(dim, n, form)
    rng = np.random.default_rng(2)
    u = rng.uniform(-1, 1, p.n)
    u[p.dirichlet] = 0
    v = rng.uniform(-1, 1, p.n)
    v[p.dirichlet] = 0
    J = O.jacobian(p, u)
    F0 = O.residual(p, u)
    errs = []
    for eps in (1e-2, 5e-3, 2.5e-3):
        errs.append(np.linalg.norm(O.residual(p, u + eps * v) - F0 - eps * (J @ v)))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5       # O(eps^2)
    # full central-difference columns on the free nodes
    Jd = J.toarray()
    h = 1e-6
    for c in np.flatnonzero(~p.dirichlet)[:6]:
        e = np.zeros(p.n)
        e[c] = h
        col = (O.residual(p, u + e) - O.residual(p, u - e)) / (2 * h)
        col[p.dirichlet] = 0
        Jc = Jd[:, c].copy()
        Jc[p.dirichlet] = 0
        assert np.abs(col - Jc).max() < 1e-6 * max(1.0, np.abs(Jc).max())


@pytest.mark.parametrize("dim,n,form", [(1, 8, O.FORM_STIFF), (2, 4, O.FORM_STIFF),
                                        (3, 2, O.FORM_STIFF), (2, 4, O.FORM_MASS)])
def test_lifted_newton_matches_reduced(dim, n, form):
    p = _small_problem(dim, n, form)
    u_red, st = O.newton(p, tol=1e-14, max_iter=40)
    u_lift, a_lift, hist = O.newton_lifted(p, tol=1e-14)
    assert np.linalg.norm(u_red - u_lift) <= 1e-12 * np.linalg.norm(u_red)
    assert np.abs(a_lift - (p.a0 + u_lift ** 2)).max() < 1e-12


# ----------------------------------------------------------------------------
# closed-form solutions
# ----------------------------------------------------------------------------
def _cardano(p_, q_):
    """Real root of t^3 + p t + q = 0 for p > 0."""
    disc = math.sqrt(q_ * q_ / 4 + p_ ** 3 / 27)
    return math.copysign(abs(-q_ / 2 + disc) ** (1 / 3), -q_ / 2 + disc) + \
        math.copysign(abs(-q_ / 2 - disc) ** (1 / 3), -q_ / 2 - disc)


def test_single_interior_node_1d():
    """n = 2, h = 1/2: F_1 = u (sum_k T_11k a_k) - d_1 = 4u + 2u^3 - d_1."""
    m = W.mesh_1d(2)
    for fval in (0.3, 7.0, -12.0):
        wl = W.Workload("t", m, np.full(3, fval), O.FORM_STIFF, None, 1.0, False, 1e-14, 0)
        p = O.build_problem(wl)
        u, st = O.newton(p, tol=1e-15, max_iter=60)
        d1 = p.d[1]
        ex = _cardano(2.0, -d1 / 2.0)          # u^3 + 2u - d1/2 = 0
        assert abs(u[1] - ex) <= 1e-14 * max(1.0, abs(ex))


def _one_node_problem(fval):
    m = W.mesh_1d(2)
    wl = W.Workload("t", m, np.full(3, fval), O.FORM_STIFF, None, 1.0, False, 1e-14, 0)
    return O.build_problem(wl)


def test_newton_damping_one_halving_by_hand():
    """Damping remark of Sec. 4 on the one free node, F(u) = 4u + 2u^3 - d1.
    f = -12 gives d1 = -6 (the interior row of M sums to h = 1/2).  From u = 0:
    F = 6, DF = 4, so the full step is u = -1.5 with F = -6 - 6.75 + 6 = -6.75,
    |F| > 6: rejected.  The halved step u = -0.75 gives F = -3 - 0.84375 + 6 =
    2.15625 <= (1 - 0.5e-4) 6: accepted.  The iteration then takes full steps
    to the root u = -1 (4(-1) + 2(-1)^3 + 6 = 0)."""
    p = _one_node_problem(-12.0)
    assert p.d[1] == -6.0
    u1, st1 = O.newton(p, tol=1e-15, max_iter=1)
    assert st1.backtracks == 1 and st1.iterations == 1
    assert u1[1] == -0.75
    assert st1.residual_norms == [6.0, 2.15625]
    u, st = O.newton(p, tol=1e-15, max_iter=60)
    assert st.status == "converged" and st.backtracks == 1
    assert abs(u[1] + 1.0) <= 1e-15
    # residual norms fall monotonically after the damped step
    h = st.residual_norms
    assert all(b < a for a, b in zip(h[1:], h[2:]) if a > 0)


@pytest.mark.parametrize("d_sq,halved", [(31.999, True), (32.0 * (1.0 - 1.5e-4), False)])
def test_newton_sufficient_decrease_constant(d_sq, halved):
    """The acceptance test ||F(u + alpha delta)|| <= (1 - 1e-4 alpha) ||F(u)||.
    From u = 0 the full step is u = d1/4 with F = d1^3/32, so the trial ratio
    |F(d1/4)| / |F(0)| is d1^2/32.  d1^2 = 31.999 gives 0.99996875: a plain
    decrease (or a constant below 3.1e-5) would accept it, the rule rejects it
    and the halved step u = d1/8 is taken.  d1^2 = 32 (1 - 1.5e-4) gives
    0.99985 <= 0.9999: accepted (a constant of 1.5e-4 or more would reject)."""
    d1 = -math.sqrt(d_sq)
    p = _one_node_problem(2.0 * d1)
    assert abs(p.d[1] - d1) <= 4e-16 * abs(d1)
    u1, st1 = O.newton(p, tol=1e-15, max_iter=1)
    assert st1.backtracks == (1 if halved else 0)
    step = d1 / 8.0 if halved else d1 / 4.0
    assert abs(u1[1] - step) <= 1e-15 * abs(step)
    ratio = st1.residual_norms[1] / st1.residual_norms[0]
    if halved:
        # the halved step: F(d1/8) = -d1/2 + d1^3/256, ratio 1/2 - d1^2/256
        assert abs(ratio - (0.5 - d_sq / 256.0)) <= 1e-14
    else:
        assert abs(ratio - d_sq / 32.0) <= 1e-14


def _thomas(a, b, c, r):
    n = len(b)
    cp = np.zeros(n)
    dp = np.zeros(n)
    cp[0] = c[0] / b[0]
    dp[0] = r[0] / b[0]
    for i in range(1, n):
        den = b[i] - a[i] * cp[i - 1]
        cp[i] = c[i] / den if i < n - 1 else 0.0
        dp[i] = (r[i] - a[i] * dp[i - 1]) / den
    x = np.zeros(n)
    x[-1] = dp[-1]
    for i in range(n - 2, -1, -1):
        x[i] = dp[i] - cp[i] * x[i + 1]
    return x


def test_sga_1d_kirchhoff_closed_form():
    """With exact quadrature the 1D SGA residual is K V(u) - d, V(u) = u + u^3/3
    (grad phi_i is constant on each cell), so u_i solves u + u^3/3 = V_i with
    V = K^{-1} d on the free nodes."""
    n = 32
    wl = W.nonlinear_diffusion_1d(n)
    p = O.build_problem(wl)
    u, st = O.sga_newton(p, tol=1e-15, max_iter=60)
    h = 1.0 / n
    nf = n - 1
    V = _thomas(np.full(nf, -1 / h), np.full(nf, 2 / h), np.full(nf, -1 / h), p.d[1:-1])
    ex = np.array([_cardano(3.0, -3.0 * v) for v in V])
    assert np.abs(u[1:-1] - ex).max() <= 1e-13 * np.abs(ex).max()


def test_egfem_p2_equals_sga():
    """Case 1: W_h = P2 describes u_h^2 exactly, so EGFEM(P2) == SGA."""
    for dim, n, form in [(1, 16, O.FORM_STIFF), (2, 6, O.FORM_STIFF), (2, 6, O.FORM_MASS)]:
        p = _small_problem(dim, n, form)
        rng = np.random.default_rng(3)
        u = rng.uniform(-1, 1, p.n)
        u[p.dirichlet] = 0
        q = O.build_problem_p2(p)
        Fs = O.sga_residual(p, u)
        assert np.abs(O.residual_p2(q, u) - Fs).max() <= 1e-13 * np.abs(Fs).max()
        Js = O.sga_jacobian(p, u)
        assert abs(O.jacobian_p2(q, u) - Js).max() <= 1e-13 * abs(Js).max()
        u1, _ = O.newton_p2(q, tol=1e-14)
        u2, _ = O.sga_newton(p, tol=1e-14)
        assert np.linalg.norm(u1 - u2) <= 1e-13 * np.linalg.norm(u2)


def test_egfem_p1_vs_sga_second_order():
    """Case 2 (P1) is an O(h^2) perturbation of SGA."""
    diffs = []
    for n in (16, 32, 64, 128):
        m = W.mesh_1d(n)
        x = m.coords[:, 0]
        wl = W.Workload("t", m, 20 * np.sin(np.pi * x) + 5, O.FORM_STIFF, None, 1.0, False, 1e-14, 0)
        p = O.build_problem(wl)
        u1, _ = O.newton(p, tol=1e-14)
        u2, _ = O.sga_newton(p, tol=1e-14)
        diffs.append(np.abs(u1 - u2).max())
    ratios = [diffs[i] / diffs[i + 1] for i in range(3)]
    assert 3.7 < ratios[-1] < 4.3 and ratios[0] < ratios[1] < ratios[2], ratios


def test_manufactured_solution_second_order():
    """u* = sin(pi x) sin(pi y) vanishes on the boundary.  For
    -div((1+u^2) grad u) = f:  f = 2 pi^2 u (1+u^2) - 2 u |grad u|^2;
    for -Laplace u + u^3 = f:  f = 2 pi^2 u + u^3.  Nodal errors decay as h^2."""
    for form in (O.FORM_STIFF, O.FORM_MASS):
        errs = []
        for n in (8, 16, 32):
            m = W.mesh_2d(n)
            x, y = m.coords[:, 0], m.coords[:, 1]
            us = np.sin(np.pi * x) * np.sin(np.pi * y)
            g2 = np.pi ** 2 * (np.cos(np.pi * x) ** 2 * np.sin(np.pi * y) ** 2 +
                               np.sin(np.pi * x) ** 2 * np.cos(np.pi * y) ** 2)
            if form == O.FORM_STIFF:
                f = 2 * np.pi ** 2 * us * (1 + us ** 2) - 2 * us * g2
                wl = W.Workload("t", m, f, form, None, 1.0, False, 1e-13, 0)
            else:
                f = 2 * np.pi ** 2 * us + us ** 3
                wl = W.Workload("t", m, f, form, None, 0.0, True, 1e-13, 0)
            p = O.build_problem(wl)
            u, st = O.newton(p, tol=1e-13)
            errs.append(np.abs(u - us).max())
        assert 3.3 < errs[0] / errs[1] < 4.7 and 3.3 < errs[1] / errs[2] < 4.7, errs


# ----------------------------------------------------------------------------
# adjoint
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("dim,n", [(2, 5), (3, 2)])
def test_adjoint_against_finite_differences(dim, n):
    rng = np.random.default_rng(7)
    m = W.structured_mesh(dim, n)
    kappa = rng.uniform(0.5, 2.0, m.n_nodes)
    f = rng.uniform(0, 10, m.n_nodes)
    u_d = rng.uniform(0, 0.2, m.n_nodes)

    def solve(fv, kv):
        wl = W.Workload("t", m, fv, O.FORM_STIFF, kv, 0.0, False, 1e-15, 0)
        p = O.build_problem(wl)
        u, _ = O.newton(p, tol=1e-15, max_iter=60)
        return p, u

    p, u = solve(f, kappa)
    lam, gf, gk = O.adjoint_gradients(p, u, u - u_d)
    # dot-product test of the transpose solve: <J v, lam> = <v, J^T lam>
    J = O.jacobian(p, u)
    v = rng.uniform(-1, 1, p.n)
    rhs = (u - u_d).copy()
    rhs[p.dirichlet] = 0
    assert abs((J @ v) @ lam - v @ rhs) < 1e-12 * max(1.0, abs(v @ rhs))
    h = 1e-6
    for vec, grad, which in ((v, gf, "f"), (rng.uniform(-1, 1, p.n), gk, "k")):
        if which == "f":
            jp = O.tracking_objective(solve(f + h * vec, kappa)[1], u_d)
            jm = O.tracking_objective(solve(f - h * vec, kappa)[1], u_d)
        else:
            jp = O.tracking_objective(solve(f, kappa + h * vec)[1], u_d)
            jm = O.tracking_objective(solve(f, kappa - h * vec)[1], u_d)
        fd = (jp - jm) / (2 * h)
        assert abs(fd - grad @ vec) <= 1e-6 * max(abs(fd), 1e-8), (which, fd, grad @ vec)


def test_elementwise_residual_equals_tensor_residual():
    """int a_h grad u_h . grad phi_i with a_h in P1 is exactly T:(u (x) a)."""
    for dim, n, form in [(1, 9, O.FORM_STIFF), (2, 7, O.FORM_STIFF), (3, 3, O.FORM_STIFF),
                         (2, 7, O.FORM_MASS)]:
        p = _small_problem(dim, n, form)
        u = np.random.default_rng(4).uniform(-1, 1, p.n)
        u[p.dirichlet] = 0
        F1 = O.residual(p, u)
        F2 = O.residual_elementwise(p, u)
        assert np.abs(F1 - F2).max() <= 1e-13 * np.abs(F1).max()
        rows = np.array([0, p.n // 3, p.n // 2, p.n - 1])
        F3 = O.residual_elementwise(p, u, rows)
        assert np.abs(F3[rows] - F1[rows]).max() <= 1e-13 * np.abs(F1).max()
        Tr = O.tensor_rows(p.coords, p.cells, form, rows)
        D = p.T.dense()
        Dr = Tr.dense()
        assert np.abs(D[rows] - Dr[rows]).max() <= 1e-15 * np.abs(D).max()


# ----------------------------------------------------------------------------
# Picard iteration (Sec. 4, Example picard_iteration)
# ----------------------------------------------------------------------------
def test_picard_single_node_recurrence():
    """n = 2, h = 1/2: the one free row of A(u) = [T . a(u)] is 4 + 2u^2, so
    the Picard iterates follow u <- d_1 / (4 + 2u^2) exactly and converge to
    the real root of 4u + 2u^3 = d_1."""
    m = W.mesh_1d(2)
    for fval in (0.3, 7.0, -12.0):
        wl = W.Workload("t", m, np.full(3, fval), O.FORM_STIFF, None, 1.0, False, 1e-14, 0)
        p = O.build_problem(wl)
        d1 = p.d[1]
        t = 0.0
        for n_it in range(1, 6):
            t = d1 / (4.0 + 2.0 * t * t)
            u, st = O.picard(p, tol=0.0, max_iter=n_it)
            assert abs(u[1] - t) <= 1e-14 * max(1.0, abs(t))
            assert u[0] == 0.0 and u[2] == 0.0
        u, st = O.picard(p, tol=1e-15, max_iter=500)
        ex = _cardano(2.0, -d1 / 2.0)
        assert st.status == "converged"
        assert abs(u[1] - ex) <= 1e-13 * max(1.0, abs(ex))


@pytest.mark.parametrize("dim,n,form", [(1, 12, O.FORM_STIFF), (2, 6, O.FORM_STIFF), (2, 5, O.FORM_MASS),
                                        (3, 3, O.FORM_STIFF)])
def test_picard_matrix_reproduces_residual(dim, n, form):
    """A(u) u - d = F(u) on the free rows (T : (u (x) a) = (T . a) u), with
    identity rows on the Dirichlet nodes."""
    p = _small_problem(dim, n, form)
    u = np.random.default_rng(4).uniform(-1, 1, p.n)
    u[p.dirichlet] = 0.0
    A = O.picard_matrix(p, u)
    r = A @ u - p.d
    F = O.residual(p, u)
    assert np.linalg.norm((r - F)[p.free]) <= 1e-13 * np.linalg.norm(p.d)
    Ad = A.toarray()
    assert np.allclose(Ad, Ad.T, rtol=0, atol=1e-14 * np.abs(Ad).max())    # symmetric
    assert np.all(Ad[np.ix_(p.dirichlet, p.dirichlet)] == np.eye(int(p.dirichlet.sum())))
    assert np.linalg.eigvalsh(Ad[np.ix_(p.free, p.free)]).min() > 0          # positive definite


@pytest.mark.parametrize("name", ["1d", "2d", "semilinear", "3d"])
def test_picard_fixed_point_is_newton_solution(name):
    wl = {"1d": lambda: W.nonlinear_diffusion_1d(64), "2d": lambda: W.nonlinear_diffusion_2d(20),
          "semilinear": lambda: W.semilinear_2d(16), "3d": lambda: W.diffusion_3d(4)}[name]()
    p = O.build_problem(wl)
    up, st = O.picard(p, tol=1e-13)
    un, _ = O.newton(p, tol=1e-14)
    assert st.status == "converged"
    assert np.linalg.norm(up - un) <= 1e-11 * np.linalg.norm(un)
    # linear convergence: the update ratios stay below one after the first step
    r = np.array(st.updates[1:-1]) / np.array(st.updates[:-2])
    assert np.all(r < 1.0)


# ----------------------------------------------------------------------------
# Burgers' equation (Sec. 5.2): convection tensor and semi-implicit steps
# ----------------------------------------------------------------------------
def test_convection_tensor_identities():
    for dim, n in [(1, 8), (2, 6), (3, 3)]:
        m = W.structured_mesh(dim, n)
        T = O.assemble_tensor(m.coords, m.cells, O.FORM_CONV)
        D = T.dense()
        assert np.abs(D - D.transpose(0, 2, 1)).max() < 1e-16             # N_ijk = N_ikj
        assert np.abs(D.sum(axis=0)).max() < 1e-14                          # sum_i grad phi_i = 0
        # sum_jk N_ijk = int sum_d d_d phi_i = 0 unless phi_i touches the boundary
        inner = m.dirichlet == 0
        assert np.abs(D.sum(axis=(1, 2))[inner]).max() < 1e-14
        # u . N:(u (x) u) = 1/3 int sum_d d_d (u^3) = 0 for u vanishing on the boundary
        rng = np.random.default_rng(7)
        u = rng.uniform(-1.0, 1.0, T.n) * inner
        c = O.contract_uv(T, u, u)
        assert abs(u @ c) < 1e-14 * np.abs(u).sum() * np.abs(c).max()
        assert np.abs(c).max() > 1e-2 * np.abs(D).max()


def test_group_matrix_closed_form():
    """N^f_ik = int phi_k (d_1 + d_2) phi_i = sum_e (sum_d d_d lambda_a) |e| / (d+1)."""
    for dim in (1, 2, 3):
        coords, cells = IRREGULAR[dim]
        sy = O.burgers_system(coords, cells, np.zeros(coords.shape[0], np.uint8), 0.1, 1.0)
        n = coords.shape[0]
        ex = np.zeros((n, n))
        for cell in cells:
            verts = [[Fraction(float(x)) for x in coords[v]] for v in cell]
            grads, vol = _exact_element(verts)
            for a in range(dim + 1):
                for c in range(dim + 1):
                    ex[cell[a], cell[c]] += float(sum(grads[a]) * vol / (dim + 1))
        assert np.abs(sy.Nf.toarray() - ex).max() < 1e-14 * np.abs(ex).max()


def test_burgers_linear_limit_eigen_decay():
    """With a tiny initial amplitude the convection term is negligible and no
    source acts, so a generalised eigenvector K v = lam M v (free rows) decays
    by the factor 1 / (1 + dt nu lam) per semi-implicit step."""
    m = W.mesh_2d(6)
    dt, nu = 0.05, 0.7
    sy = O.burgers_system(m.coords, m.cells, m.dirichlet, dt, nu)
    f = sy.free
    import scipy.linalg as sla
    lam, V = sla.eigh(sy.K.toarray()[np.ix_(f, f)], sy.M.toarray()[np.ix_(f, f)])
    for q in (0, 3, len(lam) - 1):
        v = np.zeros(m.n_nodes)
        v[f] = V[:, q]
        eps = 1e-12
        hist = O.burgers(sy, eps * v, None, 4, history=True)
        for k, uk in enumerate(hist):
            ref = eps * v / (1.0 + dt * nu * lam[q]) ** k
            assert np.abs(uk - ref).max() <= 1e-8 * np.abs(ref).max()


def test_burgers_manufactured_solution():
    """The semi-implicit EGFEM scheme converges to the paper's manufactured
    solution (nu = 1, T = 1, dt = 1e-2) at second order in h; a mistake in the
    convection term (sign, the factor 1/2, the gradient on j) is visible."""
    import dataclasses
    errs = {}
    for n in (16, 32):
        b = W.burgers_2d(n)
        sy = O.burgers_system(b.mesh.coords, b.mesh.cells, b.mesh.dirichlet, b.dt, b.nu)
        for group in (False, True):
            u = O.burgers(sy, b.u0, b.source, b.steps, group=group)
            errs[n, group] = np.linalg.norm(u - b.u_final) / np.linalg.norm(b.u_final)
        if n == 32:
            def err(N):
                u = O.burgers(dataclasses.replace(sy, N=N), b.u0, b.source, b.steps)
                return np.linalg.norm(u - b.u_final) / np.linalg.norm(b.u_final)
            T = sy.N
            assert err(dataclasses.replace(T, v=-T.v)) > 10 * errs[32, False]
            assert err(dataclasses.replace(T, v=2 * T.v)) > 10 * errs[32, False]
            assert err(dataclasses.replace(T, i=T.j, j=T.i)) > 10 * errs[32, False]
    for group in (False, True):
        assert errs[32, group] < 3e-3
        assert 3.0 < errs[16, group] / errs[32, group] < 5.0
    # interpolating u^2 onto P1 changes the result at the discretisation-error level only
    assert abs(errs[32, True] - errs[32, False]) < 0.05 * errs[32, False]


# ----------------------------------------------------------------------------
# W_h = I_k, the quadrature-point coefficient space (Case 3 of Sec. 3.1)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("dim,degree", [(1, 3), (2, 2), (3, 2)])
def test_iq_rule_exact_for_its_degree(dim, degree):
    lam, wts = O.iq_rule(dim)
    assert abs(wts.sum() - 1.0) < 1e-15 and np.allclose(lam.sum(axis=1), 1.0, atol=1e-15)
    for alpha in itertools.product(range(degree + 1), repeat=dim + 1):
        if sum(alpha) > degree:
            continue
        num = np.sum(wts * np.prod(lam ** np.array(alpha), axis=1))      # relative to |e|
        ex = float(_int_monomial(alpha, Fraction(1), dim))
        assert abs(num - ex) < 1e-15, (alpha, num, ex)
    # and not exact one degree higher (a plausible mistake in the points shows here)
    hi = [a for a in itertools.product(range(degree + 2), repeat=dim + 1) if sum(a) == degree + 1]
    errs = [abs(np.sum(wts * np.prod(lam ** np.array(a), axis=1)) - float(_int_monomial(a, Fraction(1), dim)))
            for a in hi]
    assert max(errs) > 1e-6


def test_egfem_iq_equals_sga_and_p2():
    """With a rule exact for (a0 + u_h^2) grad u_h . grad phi_i the quadrature
    space reproduces the standard Galerkin approach, like W_h = P2."""
    for dim, n in [(1, 16), (2, 6), (3, 3)]:
        p = _small_problem(dim, n, O.FORM_STIFF)
        q = O.build_problem_iq(p)
        rng = np.random.default_rng(9)
        u = rng.uniform(-1, 1, p.n)
        u[p.dirichlet] = 0
        Fs = O.sga_residual(p, u)
        assert np.abs(O.residual_p2(q, u) - Fs).max() <= 1e-13 * np.abs(Fs).max()
        Js = O.sga_jacobian(p, u)
        assert abs(O.jacobian_p2(q, u) - Js).max() <= 1e-13 * abs(Js).max()
        u1, _ = O.newton_p2(q, tol=1e-14)
        u2, _ = O.newton_p2(O.build_problem_p2(p), tol=1e-14)
        assert np.linalg.norm(u1 - u2) <= 1e-13 * np.linalg.norm(u2)
        # the quadrature functionals sum to the element volumes
        T, Wsp = O.tensor_iq(p.coords, p.cells, O.FORM_STIFF)
        assert Wsp.n_w == p.cells.shape[0] * Wsp.lam.shape[0]
        assert np.allclose(np.asarray(Wsp.Pi.sum(axis=1)).ravel(), 1.0)


# ----------------------------------------------------------------------------
# W_h = P0 with the gradient interpolation (p-Laplace, minimal surface)
# ----------------------------------------------------------------------------
def test_p0_tensor_is_element_stiffness():
    """T_ijk = K^{e_k}_ij: contracting with a = 1 gives the stiffness matrix, and
    the per-cell slices are the exact rational element stiffness matrices."""
    for dim in (1, 2, 3):
        coords, cells = IRREGULAR[dim]
        T = O.tensor_p0(coords, cells, drop_rel=0.0)
        K = O.assemble_stiffness(coords, cells).toarray()
        n = coords.shape[0]
        A = np.zeros((n, n))
        np.add.at(A, (T.i, T.j), T.v)
        assert np.abs(A - K).max() < 1e-14 * np.abs(K).max()
        for e, cell in enumerate(cells):
            verts = [[Fraction(float(x)) for x in coords[v]] for v in cell]
            grads, vol = _exact_element(verts)
            sel = T.k == e
            for i, j, v in zip(T.i[sel], T.j[sel], T.v[sel]):
                a, b = list(cell).index(i), list(cell).index(j)
                ex = float(vol * sum(grads[a][r] * grads[b][r] for r in range(dim)))
                assert abs(v - ex) <= 1e-14 * abs(ex) + 1e-17


def test_plaplace_1d_exact_fluxes():
    """1D p-Laplace, source 1, zero boundary values: the discrete equations fix the
    element fluxes a(u'_e) u'_e = 1/2 - x_mid(e) exactly (a telescoping sum with the
    loads int phi_i = h), whatever the nonlinearity."""
    m = W.mesh_1d(40)
    for pp in (1.5, 1.8):
        wl = W.GradientWorkload("t", m, np.ones(m.n_nodes), pp, 0.0, 1.0, (pp - 2.0) / 2.0, None)
        P = O.build_grad_problem(wl)
        u, it = O.picard_grad(P, tol=1e-14)
        z = O.grad_interp(P, u)[:, 0]
        flux = O.grad_coef(P, u) * z
        xm = m.coords[m.cells].mean(axis=1)[:, 0]
        assert np.abs(flux - (0.5 - xm)).max() < 1e-12
    # q = 0 is the linear problem: one solve with the stiffness matrix
    wl = W.GradientWorkload("t", m, np.ones(m.n_nodes), 2.0, 1.0, 1.0, 0.0, None)
    P = O.build_grad_problem(wl)
    u, it = O.picard_grad(P, tol=1e-14)
    assert it <= 2
    x = m.coords[:, 0]
    assert np.abs(u - 0.5 * x * (1 - x)).max() < 1e-14        # P1 is nodally exact in 1D


def test_plaplace_disk_converges_to_exact_solution():
    """p = 3/2 on the unit disk (the paper's example): the EGFEM(P0) fixed point
    approaches the radial exact solution at second order."""
    errs = []
    for n in (8, 16, 32):
        wl = W.plaplace_disk(n)
        P = O.build_grad_problem(wl)
        u, it = O.picard_grad(P, tol=1e-12)
        assert np.linalg.norm(O.residual_grad(P, u)) <= 1e-11 * np.linalg.norm(P.d[P.free])
        errs.append(np.linalg.norm(u - wl.exact) / np.linalg.norm(wl.exact))
    assert errs[2] < 2e-3
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


def test_gradient_newton_jacobian_and_fixed_point():
    """The analytic Jacobian of the gradient nonlinearity passes the Taylor test
    (remainder O(eps^2)), and damped Newton reaches the Picard fixed point."""
    cases = [W.GradientWorkload("ms", W.mesh_2d(16), np.ones(17 * 17), 0.0, 1.0, 1.0, -0.5, None),
             W.plaplace_disk(16)]
    for wl in cases:
        P = O.build_grad_problem(wl)
        u, _ = O.picard_grad(P, tol=1e-12)
        v = np.random.default_rng(3).uniform(-1, 1, P.n)
        v[P.dirichlet] = 0.0
        J = O.jacobian_grad(P, u)
        F0 = O.residual_grad(P, u)
        rem = [np.linalg.norm(O.residual_grad(P, u + e * v) - F0 - e * (J @ v)) for e in (1e-3, 1e-4, 1e-5)]
        assert rem[1] < rem[0] / 30 and rem[2] < rem[1] / 60, rem
        assert abs(J - J.T).max() <= 1e-13 * abs(J).max()            # symmetric
        un, st = O.newton_grad(P, tol=1e-13)
        assert st.status == "converged" and st.iterations <= 10
        assert np.linalg.norm(un - u) <= 1e-10 * np.linalg.norm(u)


def test_burgers_egfem_p2_is_exact():
    """With W_h = P2 the group formulation interpolates u^2 without error
    ((Pi_u u)^2 is u_h^2 in P2), so N^f_P2 (Pi_u u)^2 = N:(u (x) u) and the
    EGFEM(P2) steps reproduce the tensor formulation, unlike the P1 group one."""
    for m in (W.mesh_1d(9), W.mesh_2d(7), W.mesh_3d(3)):
        T = O.assemble_tensor(m.coords, m.cells, O.FORM_CONV)
        Nf2, W2 = O.burgers_group_p2(m.coords, m.cells)
        u = np.random.default_rng(1).uniform(-1, 1, m.n_nodes)
        pu = W2.Pi @ u
        c = O.contract_uv(T, u, u)
        assert np.abs(Nf2 @ (pu * pu) - c).max() <= 1e-14 * np.abs(c).max()
    b = W.burgers_2d(16)
    sy = O.burgers_system(b.mesh.coords, b.mesh.cells, b.mesh.dirichlet, b.dt, b.nu)
    ut = O.burgers(sy, b.u0, b.source, b.steps)
    u2 = O.burgers(sy, b.u0, b.source, b.steps, group_p2=O.burgers_group_p2(b.mesh.coords, b.mesh.cells))
    ug = O.burgers(sy, b.u0, b.source, b.steps, group=True)
    assert np.linalg.norm(u2 - ut) <= 1e-13 * np.linalg.norm(ut)
    assert np.linalg.norm(ug - ut) > 1e-6 * np.linalg.norm(ut)


def test_burgers_egfem_iq_one_cell_by_hand():
    """One 1D cell [0, h] with the 2-point Gauss rule: N^f_{i,q} = w_q h phi_i' =
    -1/2, +1/2 for i = 0, 1 at both points, and with u = (a, b) the group value
    sum_q N^f_{1,q} u(x_q)^2 is int_0^h u^2 / h = (a^2 + ab + b^2) / 3."""
    h = 0.3
    coords = np.array([[0.0], [h]])
    cells = np.array([[0, 1]])
    Nf, Wsp = O.burgers_group_iq(coords, cells)
    assert Wsp.n_w == 2
    assert np.allclose(Nf.toarray(), [[-0.5, -0.5], [0.5, 0.5]], rtol=0, atol=1e-15)
    a, b = 0.7, -1.9
    pu = Wsp.Pi @ np.array([a, b])
    c = Nf @ (pu * pu)
    assert abs(c[1] - (a * a + a * b + b * b) / 3.0) <= 1e-15
    assert abs(c[0] + c[1]) <= 1e-15


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_burgers_egfem_iq_matches_exact_tensor(dim):
    """The points' rule integrates the quadratic (P1 u)^2 times the constant
    gradient sum exactly (degree 3 in 1D, 2 in 2D and 3D), so N^f_I (Pi_u u)^2
    equals the exact rational convection tensor contracted with u (x) u, and
    the points of one cell carry weights summing to |e| sum_d d_d phi_i."""
    coords, cells = IRREGULAR[dim]
    n = coords.shape[0]
    Te = _exact_tensor(coords, cells, O.FORM_CONV)
    u = np.random.default_rng(31).uniform(-1, 1, n)
    c_exact = np.zeros(n)
    for (i, j, k), v in Te.items():
        c_exact[i] += float(v) * u[j] * u[k]
    Nf, Wsp = O.burgers_group_iq(coords, cells)
    pu = Wsp.Pi @ u
    c = Nf @ (pu * pu)
    assert np.abs(c - c_exact).max() <= 1e-14 * np.abs(c_exact).max()
    Q = Wsp.lam.shape[0]
    Nd = Nf.toarray()
    for e, cell in enumerate(cells):
        verts = [[Fraction(float(x)) for x in coords[v]] for v in cell]
        grads, vol = _exact_element(verts)
        for a, i in enumerate(cell):
            want = float(vol * sum(grads[a]))
            got = Nd[i, e * Q:(e + 1) * Q].sum()
            assert abs(got - want) <= 1e-14 * max(1.0, abs(want)), (e, a)


def test_burgers_egfem_iq_steps_equal_tensor_formulation():
    """Exactness carries to the time steps: EGFEM(I_k) reproduces the tensor
    formulation, while the P1 group formulation differs."""
    b = W.burgers_2d(16)
    sy = O.burgers_system(b.mesh.coords, b.mesh.cells, b.mesh.dirichlet, b.dt, b.nu)
    ut = O.burgers(sy, b.u0, b.source, b.steps)
    ui = O.burgers(sy, b.u0, b.source, b.steps, group_p2=O.burgers_group_iq(b.mesh.coords, b.mesh.cells))
    ug = O.burgers(sy, b.u0, b.source, b.steps, group=True)
    assert np.linalg.norm(ui - ut) <= 1e-13 * np.linalg.norm(ut)
    assert np.linalg.norm(ug - ut) > 1e-6 * np.linalg.norm(ut)
