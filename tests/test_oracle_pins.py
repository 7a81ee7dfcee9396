"""Pins of the CPU oracle against mathematics that does not come from it.

Each test fixes one oracle routine with something independent: dense linear
algebra built from the LDU definition (paper Sec. 2.1), closed-form
eigenpairs of the 7-point operator, finite termination of CG, the greedy
characterisation of handshake matching, the dense Galerkin product, and
finite differences for the adjoint.  CPU only.
"""
import numpy as np
import pytest

import oracle as O
from meshgen import (assemble_diag, box_case, box_faces, c3_assembly_inputs,
                     config_case, random_order, relabel)
from meshgen.boxes import LduCase, c3_spacing
from tests.dense_ref import (closed_form_1d, dense, dense_case,
                             galerkin_ldu, greedy_matching,
                             pairwise_aggregation, prolongation, strength2,
                             tie_key)


def _perm_case(case, seed):
    return relabel(case, random_order(case.n_cells, np.random.default_rng(seed)))


# ---------------------------------------------------------------- generators

@pytest.mark.parametrize("shape", [(4, 4, 4), (3, 2, 5), (1, 4, 3), (7, 1, 1)])
def test_box_face_count_and_order(shape):
    nx, ny, nz = shape
    own, nb, _ = box_faces(nx, ny, nz)
    assert own.size == (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)
    assert np.all(own < nb)
    key = own.astype(np.int64) * (nx * ny * nz) + nb
    assert np.all(np.diff(key) > 0)
    assert O.validate(nx * ny * nz, own, nb) == O.OK


def test_config_face_counts():
    # 3 n^2 (n-1) internal faces for an n^3 box
    for n, f in [(32, 95232), (128, 6242304), (200, 23880000), (256, 50135040),
                 (100, 2970000)]:
        assert 3 * n * n * (n - 1) == f


def test_neumann_zero_row_sum_and_symmetry():
    c = config_case("c2", n=8)
    A = dense_case(c)
    assert np.allclose(A, A.T, rtol=0, atol=0)
    assert np.max(np.abs(A.sum(1))) <= 1e-14 * np.max(np.abs(c.diag))
    assert np.all(c.diag < 0)
    assert abs(c.rhs[0].sum()) < 1e-12
    assert O.validate(c.n_cells, c.owner, c.neighbour, c.diag, c.upper,
                      c.lower) == O.OK


def test_c3_grading_spans_four_decades():
    dx, dz = c3_spacing(200)
    assert dx / dz.min() == pytest.approx(100.0)
    assert np.sum(dz < dx) == 95
    ax = dz  # a_x = a_y = dz_k
    az = dx * dx / (0.5 * (dz[:-1] + dz[1:]))
    lo, hi = min(ax.min(), az.min()), max(ax.max(), az.max())
    assert 3.9 < np.log10(hi / lo) < 4.1


# ---------------------------------------------------------------- Amul / Tmul

def _tiny_cases():
    out = []
    for seed in range(3):
        c = box_case(4, 3, 5, coeff="lognormal", dirichlet_x0=1.5, seed=seed)
        out.append(_perm_case(c, 100 + seed))
        out.append(_perm_case(box_case(3, 4, 2, coeff="lognormal", nonsym=0.7,
                                       seed=seed), 200 + seed))
    return out


@pytest.mark.parametrize("idx", range(6))
def test_amul_tmul_match_dense(idx):
    c = _tiny_cases()[idx]
    A = O.Ldu.from_case(c)
    D = dense_case(c)
    x = np.random.default_rng(idx).standard_normal(c.n_cells)
    scale = np.abs(D) @ np.abs(x)
    assert np.all(np.abs(O.amul(A, x) - D @ x) <= 1e-15 * 8 * scale)
    assert np.all(np.abs(O.tmul(A, x) - D.T @ x) <= 1e-15 * 8 * (np.abs(D.T) @ np.abs(x)))


@pytest.mark.parametrize("kind", ["neumann", "dirichlet0", "dirichlet_node"])
def test_amul_closed_form_eigenpairs(kind):
    nx, ny, nz, h = 5, 4, 6, 0.25
    own, nb, _ = box_faces(nx, ny, nz)
    n = nx * ny * nz
    a = np.full(own.size, 1.0 / h ** 2)
    ix = np.arange(n) % nx
    iy = (np.arange(n) // nx) % ny
    iz = np.arange(n) // (nx * ny)
    if kind == "dirichlet_node":
        diag = np.full(n, -6.0 / h ** 2)
        kinds = ("dirichlet_node",) * 3
    else:
        ab = np.where(ix == 0, 2.0 / h ** 2, 0.0) if kind == "dirichlet0" else None
        diag = assemble_diag(n, own, nb, a, a, ab)
        kinds = (kind, "neumann", "neumann")
    A = O.Ldu(n, own, nb, diag, a, a)
    lx, Vx = closed_form_1d(nx, h, kinds[0])
    ly, Vy = closed_form_1d(ny, h, kinds[1])
    lz, Vz = closed_form_1d(nz, h, kinds[2])
    for kx, ky, kz in [(0, 0, 0), (1, 2, 3), (4, 3, 5), (2, 0, 1)]:
        v = Vx[ix, kx] * Vy[iy, ky] * Vz[iz, kz]
        lam = lx[kx] + ly[ky] + lz[kz]
        r = O.amul(A, v) + lam * v
        assert np.linalg.norm(r) <= 1e-13 * (6 / h ** 2) * np.linalg.norm(v)


def test_amul_f32_error_bound():
    c = _perm_case(box_case(6, 5, 4, coeff="lognormal", sigma=1.0,
                            dirichlet_x0=2.0, seed=7), 9)
    A = O.Ldu.from_case(c)
    D = dense_case(c)
    x = np.random.default_rng(3).uniform(-1, 1, c.n_cells)
    y32 = O.amul_f32(A, x.astype(np.float32)).astype(np.float64)
    y64 = D @ x
    # fp32 rounding of A, x, each product and each of <= 6 additions
    bound = 10 * 2.0 ** -24 * (np.abs(D) @ np.abs(x))
    assert np.all(np.abs(y32 - y64) <= bound)
    assert np.linalg.norm(y32 - y64) / np.linalg.norm(y64) <= 1e-5


# ---------------------------------------------------------------- validation

def test_validate_rejects_bad_addressing():
    own, nb, _ = box_faces(3, 3, 1)
    n = 9
    d = -np.ones(n)
    u = np.ones(own.size)
    assert O.validate(n, own, nb, d, u, u) == O.OK
    bad = nb.copy(); bad[2] = own[2]
    assert O.validate(n, own, bad, d, u, u) == O.ERR_ADDR  # owner >= neighbour
    bad = nb.copy(); bad[-1] = n
    assert O.validate(n, own, bad, d, u, u) == O.ERR_ADDR  # out of range
    assert O.validate(n, own[::-1].copy(), nb[::-1].copy(), d, u, u) == O.ERR_ADDR
    dup_o = np.concatenate([own[:3], own[2:3], own[3:]])
    dup_n = np.concatenate([nb[:3], nb[2:3], nb[3:]])
    uu = np.ones(dup_o.size)
    assert O.validate(n, dup_o, dup_n, d, uu, uu) == O.ERR_ADDR  # duplicate
    dn = d.copy(); dn[4] = np.nan
    assert O.validate(n, own, nb, dn, u, u) == O.ERR_NAN


# ---------------------------------------------------------------- PCG

@pytest.mark.parametrize("idx", [0, 2, 4])
def test_pcg_matches_dense_solve(idx):
    c = _tiny_cases()[idx]
    A = O.Ldu.from_case(c)
    D = dense_case(c)
    b = c.rhs[0]
    r = O.pcg(A, b, tol=1e-14, max_iter=1000)
    xd = np.linalg.solve(D, b)
    assert r.status == O.OK
    assert np.linalg.norm(r.x - xd) <= 1e-11 * np.linalg.norm(xd)
    assert r.true_residual <= 1e-14
    assert r.history[0] == pytest.approx(1.0)  # x0 = 0


def _node_dirichlet_box(nx, ny, nz, h):
    own, nb, _ = box_faces(nx, ny, nz)
    n = nx * ny * nz
    a = np.full(own.size, 1.0 / h ** 2)
    diag = np.full(n, -6.0 / h ** 2)
    return n, own, nb, diag, a


def _eigvec(nx, ny, nz, h, k):
    n = nx * ny * nz
    ix = np.arange(n) % nx
    iy = (np.arange(n) // nx) % ny
    iz = np.arange(n) // (nx * ny)
    lx, Vx = closed_form_1d(nx, h, "dirichlet_node")
    ly, Vy = closed_form_1d(ny, h, "dirichlet_node")
    lz, Vz = closed_form_1d(nz, h, "dirichlet_node")
    v = Vx[ix, k[0]] * Vy[iy, k[1]] * Vz[iz, k[2]]
    return v, lx[k[0]] + ly[k[1]] + lz[k[2]]


@pytest.mark.parametrize("m", [1, 2, 3])
def test_cg_finite_termination(m):
    """Unpreconditioned CG on b = sum of m eigenvectors with distinct
    eigenvalues converges in exactly m iterations."""
    nx, ny, nz, h = 6, 5, 7, 1.0
    n, own, nb, diag, a = _node_dirichlet_box(nx, ny, nz, h)
    A = O.Ldu(n, own, nb, diag, a, a)
    ks = [(0, 0, 0), (2, 1, 3), (5, 4, 6)][:m]
    b = sum((j + 1.0) * _eigvec(nx, ny, nz, h, k)[0] for j, k in enumerate(ks))
    r = O.pcg(A, b, tol=1e-10, max_iter=50, precond=False)
    assert r.status == O.OK and r.iterations == m


@pytest.mark.parametrize("m", [1, 2, 3])
def test_pcg_diagonal_finite_termination(m):
    """A = S B S with B of constant diagonal beta: the diagonally
    preconditioned operator diag(A)^-1 A has eigenvectors S^-1 v_k, so
    PCG-diag with b = beta S sum c_k v_k terminates in exactly m iterations.
    A preconditioner applied on the wrong side or not at all fails this."""
    nx, ny, nz, h = 6, 5, 7, 1.0
    n, own, nb, diag, a = _node_dirichlet_box(nx, ny, nz, h)
    s = np.exp(0.4 * np.random.default_rng(11).standard_normal(n))
    up = s[own] * a * s[nb]
    dA = diag * s * s
    A = O.Ldu(n, own, nb, dA, up, up)
    ks = [(0, 0, 0), (2, 1, 3), (5, 4, 6)][:m]
    v = sum((j + 1.0) * _eigvec(nx, ny, nz, h, k)[0] for j, k in enumerate(ks))
    b = -6.0 * s * v
    r = O.pcg(A, b, tol=1e-10, max_iter=50, precond=True)
    assert r.status == O.OK and r.iterations == m
    r0 = O.pcg(A, b, tol=1e-10, max_iter=50, precond=False)
    assert r0.iterations > m


def test_cg_iteration_bound():
    """CG iterations <= 1/2 sqrt(kappa) ln(2/tol) (Chebyshev bound)."""
    nx = ny = nz = 12
    h = 1.0
    n, own, nb, diag, a = _node_dirichlet_box(nx, ny, nz, h)
    A = O.Ldu(n, own, nb, diag, a, a)
    lmin = _eigvec(nx, ny, nz, h, (0, 0, 0))[1]
    lmax = _eigvec(nx, ny, nz, h, (nx - 1, ny - 1, nz - 1))[1]
    kappa = lmax / lmin
    b = np.random.default_rng(0).standard_normal(n)
    tol = 1e-8
    r = O.pcg(A, b, tol=tol, max_iter=5000, precond=False)
    # the bound is on the A-norm error; the residual picks up sqrt(kappa)
    bound = 0.5 * np.sqrt(kappa) * np.log(2 * np.sqrt(kappa) / tol)
    assert r.status == O.OK and r.iterations <= np.ceil(bound)


def test_c1_manufactured_solution():
    c = config_case("c1")
    A = O.Ldu.from_case(c)
    r = O.pcg(A, c.rhs[0], tol=1e-8)
    p = c.meta["p_exact"]
    # kappa of the c1 operator from its closed-form spectrum
    h = c.meta["h"]
    lx, _ = closed_form_1d(32, h, "dirichlet0")
    ln, _ = closed_form_1d(32, h, "neumann")
    kappa = (lx.max() + 2 * ln.max()) / lx.min()
    assert 4900 < kappa < 5050
    assert r.status == O.OK and r.true_residual <= 1e-8
    assert np.linalg.norm(r.x - p) <= kappa * 1e-8 * np.linalg.norm(p)


def test_pcg_edge_cases():
    c = box_case(4, coeff="lognormal", dirichlet_x0=1.0, seed=1)
    A = O.Ldu.from_case(c)
    r = O.pcg(A, np.zeros(c.n_cells), x0=np.ones(c.n_cells))
    assert r.status == O.OK and r.iterations == 0 and np.all(r.x == 0)
    r = O.pcg(A, c.rhs[0], max_iter=1)
    assert r.status == O.NOT_CONVERGED and r.iterations == 1
    # warm start from the solution: converged with zero iterations
    xs = np.linalg.solve(dense_case(c), c.rhs[0])
    r = O.pcg(A, c.rhs[0], x0=xs, tol=1e-8)
    assert r.status == O.OK and r.iterations == 0


def test_pcg_singular_consistent():
    c = _perm_case(box_case(5, 4, 3, coeff="lognormal", seed=4), 5)
    A = O.Ldu.from_case(c)
    D = dense_case(c)
    r = O.pcg(A, c.rhs[0], tol=1e-13, max_iter=2000)
    xd = np.linalg.pinv(D) @ c.rhs[0]
    d = (r.x - r.x.mean()) - (xd - xd.mean())
    assert r.status == O.OK
    assert np.linalg.norm(d) <= 1e-10 * np.linalg.norm(xd)


# ---------------------------------------------------------------- agglomeration

def _match_cases():
    return [
        _perm_case(box_case(6, 5, 4, coeff="lognormal", dirichlet_x0=1.0, seed=1), 3),
        box_case(7, 6, 5, coeff="lognormal", seed=2),
        box_case(5, 5, 5, coeff="uniform"),  # all weights tie: tie keys decide
        _perm_case(box_case(4, 6, 3, coeff="lognormal", nonsym=0.5, seed=3), 8),
    ]


@pytest.mark.parametrize("idx", range(4))
def test_matching_equals_greedy(idx):
    c = _match_cases()[idx]
    g = O.Gamg(O.Ldu.from_case(c), n_coarsest=2, max_levels=2,
               match_rounds=100000)
    L = g.level(0)
    ref = greedy_matching(c.n_cells, c.owner, c.neighbour, c.upper, c.lower, c.diag)
    assert np.array_equal(L.partner, ref)


@pytest.mark.parametrize("idx", range(4))
def test_leftovers_and_numbering(idx):
    c = _match_cases()[idx]
    g = O.Gamg(O.Ldu.from_case(c), n_coarsest=2, max_levels=2,
               match_rounds=100000)
    L = g.level(0)
    n = c.n_cells
    nbrs = [[] for _ in range(n)]
    ws = strength2(c.owner, c.neighbour, c.upper, c.lower, c.diag)
    for f in range(c.n_faces):
        i, j = int(c.owner[f]), int(c.neighbour[f])
        w = ws[f]
        nbrs[i].append((j, w))
        nbrs[j].append((i, w))
    p = L.partner
    for i in range(n):
        if p[i] >= 0:
            assert p[p[i]] == i and L.join[i] == -1
            continue
        # maximal matching: no unmatched neighbour survives
        assert all(p[j] >= 0 for j, _ in nbrs[i])
        if nbrs[i]:
            best = max(nbrs[i], key=lambda t: (t[1], tie_key(i, t[0]), -t[0]))
            assert L.join[i] == best[0]
        else:
            assert L.join[i] == -1
    # seeds ranked by cell index; pairs share an aggregate; leftovers follow
    seeds = [i for i in range(n)
             if (p[i] >= 0 and i < p[i]) or (p[i] < 0 and L.join[i] < 0)]
    rank = {s: k for k, s in enumerate(seeds)}
    for i in range(n):
        if p[i] >= 0:
            assert L.agg[i] == rank[min(i, p[i])]
        elif L.join[i] < 0:
            assert L.agg[i] == rank[i]
        else:
            assert L.agg[i] == L.agg[L.join[i]]
    assert g.level(1).n == len(seeds)


@pytest.mark.parametrize("idx", range(4))
def test_galerkin_equals_dense_ptap(idx):
    c = _match_cases()[idx]
    g = O.Gamg(O.Ldu.from_case(c), n_coarsest=3, max_levels=50)
    assert g.n_levels >= 3
    for l in range(g.n_levels - 1):
        F, Cl = g.level(l), g.level(l + 1)
        Af = dense(F.n, F.owner, F.neighbour, F.diag, F.upper, F.lower)
        P = prolongation(F.agg, Cl.n)
        Ac = dense(Cl.n, Cl.owner, Cl.neighbour, Cl.diag, Cl.upper, Cl.lower)
        ref = P.T @ Af @ P
        assert np.allclose(Ac, ref, rtol=0, atol=1e-14 * np.abs(ref).max())
        # pattern: exactly the nonzero off-diagonal pairs, upper-triangular order
        assert O.validate(Cl.n, Cl.owner, Cl.neighbour) == O.OK
        off = (P.T @ (np.abs(Af) > 0) @ P) > 0
        np.fill_diagonal(off, False)
        assert 2 * Cl.nf == off.sum()
        if np.allclose(c.upper, c.lower):
            assert np.array_equal(Cl.upper, Cl.lower)
        if c.singular:
            assert np.max(np.abs(Ac.sum(1))) <= 1e-13 * np.abs(Ac).max()


def test_coarsening_stops():
    c = box_case(9, 8, 7, coeff="lognormal", dirichlet_x0=1.0, seed=5)
    g = O.Gamg(O.Ldu.from_case(c), n_coarsest=20)
    sizes = [g.level(l).n for l in range(g.n_levels)]
    assert sizes[-1] <= 20 and all(a > b for a, b in zip(sizes, sizes[1:]))
    g1 = O.Gamg(O.Ldu.from_case(c), n_coarsest=10 ** 6)
    assert g1.n_levels == 1
    # a diagonal matrix cannot coarsen: one level
    d = O.Ldu(10, np.zeros(0, np.int32), np.zeros(0, np.int32), -np.ones(10),
              np.zeros(0), np.zeros(0))
    assert O.Gamg(d, n_coarsest=2).n_levels == 1


# ---------------------------------------------------------------- V-cycle

def _two_level(seed=0):
    c = box_case(5, 4, 3, coeff="lognormal", dirichlet_x0=1.0, seed=seed)
    g = O.Gamg(O.Ldu.from_case(c), n_coarsest=40, max_levels=2)
    assert g.n_levels == 2
    F, Cl = g.level(0), g.level(1)
    A = dense_case(c)
    P = prolongation(F.agg, Cl.n)
    return c, g, A, P


def test_vcycle_two_level_exact_coarse():
    c, g, A, P = _two_level()
    r = np.random.default_rng(1).standard_normal(c.n_cells)
    Ac = P.T @ A @ P
    ref = P @ np.linalg.solve(Ac, P.T @ r)
    e = g.vcycle(r, n_pre=0, n_post=0, scale=False)
    assert np.linalg.norm(e - ref) <= 1e-8 * np.linalg.norm(ref)
    # with an exact coarse solve the energy-optimal scaling factor is 1
    e2 = g.vcycle(r, n_pre=0, n_post=0, scale=True)
    assert np.linalg.norm(e2 - ref) <= 1e-8 * np.linalg.norm(ref)


def test_vcycle_two_level_dense_formula():
    c, g, A, P = _two_level(3)
    r = np.random.default_rng(2).standard_normal(c.n_cells)
    w = 0.75
    Dinv = 1.0 / np.diag(A)
    Ac = P.T @ A @ P
    e = w * Dinv * r                       # sweep 1 from zero
    e = e + w * Dinv * (r - A @ e)         # sweep 2
    t = r - A @ e
    cc = P @ np.linalg.solve(Ac, P.T @ t)
    s = (cc @ t) / (cc @ (A @ cc))
    e = e + s * cc
    for _ in range(2):
        e = e + w * Dinv * (r - A @ e)
    got = g.vcycle(r, n_pre=2, n_post=2, omega=w, scale=True)
    assert np.linalg.norm(got - e) <= 1e-8 * np.linalg.norm(e)


def test_vcycle_is_symmetric_without_scaling():
    c = box_case(7, 6, 5, coeff="lognormal", dirichlet_x0=1.0, seed=9)
    g = O.Gamg(O.Ldu.from_case(c), n_coarsest=10)
    assert g.n_levels >= 3
    rng = np.random.default_rng(4)
    u, v = rng.standard_normal((2, c.n_cells))
    Vu = g.vcycle(u, scale=False)
    Vv = g.vcycle(v, scale=False)
    assert abs(u @ Vv - v @ Vu) <= 1e-8 * np.linalg.norm(u) * np.linalg.norm(Vv)
    # linear: V(u + 2v) = V(u) + 2 V(v)
    Vw = g.vcycle(u + 2 * v, scale=False)
    assert np.linalg.norm(Vw - Vu - 2 * Vv) <= 1e-8 * np.linalg.norm(Vw)


def test_gamg_converges_to_dense_solution():
    c = _perm_case(box_case(8, 7, 6, coeff="lognormal", dirichlet_x0=1.0,
                            seed=12), 13)
    g = O.Gamg(O.Ldu.from_case(c), n_coarsest=10)
    r = g.solve(c.rhs[0], tol=1e-12, max_cycles=500)
    xd = np.linalg.solve(dense_case(c), c.rhs[0])
    assert r.status == O.OK and r.true_residual <= 1e-12
    assert np.linalg.norm(r.x - xd) <= 1e-10 * np.linalg.norm(xd)
    # the residual falls monotonically
    assert np.all(np.diff(r.history) < 0)


def test_gamg_singular_modulo_constant():
    c = _perm_case(box_case(7, 6, 5, coeff="lognormal", seed=14), 15)
    g = O.Gamg(O.Ldu.from_case(c), n_coarsest=10)
    r = g.solve(c.rhs[0], tol=1e-11, max_cycles=500)
    xd = np.linalg.pinv(dense_case(c)) @ c.rhs[0]
    d = (r.x - r.x.mean()) - (xd - xd.mean())
    assert r.status == O.OK
    assert np.linalg.norm(d) <= 1e-9 * np.linalg.norm(xd)


def test_gamg_transpose_nonsymmetric():
    c = _perm_case(box_case(6, 5, 4, coeff="lognormal", nonsym=0.6, seed=16), 17)
    g = O.Gamg(O.Ldu.from_case(c), n_coarsest=10)
    D = dense_case(c)
    b = c.rhs[0]
    r = g.solve(b, tol=1e-12, max_cycles=500, transpose=True)
    xd = np.linalg.solve(D.T, b)
    assert r.status == O.OK
    assert np.linalg.norm(r.x - xd) <= 1e-10 * np.linalg.norm(xd)
    rf = g.solve(b, tol=1e-12, max_cycles=500)
    assert np.linalg.norm(rf.x - np.linalg.solve(D, b)) <= 1e-10 * np.linalg.norm(xd)


# ---------------------------------------------------------------- mixed precision

def test_mixed_pcg_refines_to_fp64_solution():
    c = _perm_case(box_case(8, 7, 6, coeff="lognormal", dirichlet_x0=1.0,
                            seed=18), 19)
    A = O.Ldu.from_case(c)
    xd = np.linalg.solve(dense_case(c), c.rhs[0])
    r = O.pcg_mixed(A, c.rhs[0], tol=1e-12)
    assert r.status == O.OK and r.true_residual <= 1e-12
    assert np.linalg.norm(r.x - xd) <= 1e-10 * np.linalg.norm(xd)
    # each refinement gains about the inner tolerance
    assert r.iterations <= 6


def test_mixed_gamg_refines_to_fp64_solution():
    c = _perm_case(box_case(8, 7, 6, coeff="lognormal", dirichlet_x0=1.0,
                            seed=20), 21)
    g = O.Gamg(O.Ldu.from_case(c), n_coarsest=10)
    xd = np.linalg.solve(dense_case(c), c.rhs[0])
    r = g.solve_mixed(c.rhs[0], tol=1e-12)
    assert r.status == O.OK and r.true_residual <= 1e-12
    assert np.linalg.norm(r.x - xd) <= 1e-10 * np.linalg.norm(xd)
    r64 = g.solve(c.rhs[0], tol=1e-12)
    # an FP32 V-cycle reduces the residual about as well as an FP64 one
    assert abs(r.iterations - r64.iterations) <= 3


# ---------------------------------------------------------------- adjoint

def _adjoint_setup(seed=22):
    c = box_case(5, 4, 4, coeff="lognormal", dirichlet_x0=2.0, seed=seed)
    a = c.upper.copy()
    ab = np.where(np.arange(c.n_cells) % 5 == 0, 2.0, 0.0)
    xt = np.random.default_rng(seed + 1).standard_normal(c.n_cells)
    return c, a, ab, xt


def _loss(c, a, ab, xt):
    d = assemble_diag(c.n_cells, c.owner, c.neighbour, a, a, ab)
    A = O.Ldu(c.n_cells, c.owner, c.neighbour, d, a, a)
    r = O.pcg(A, c.rhs[0], tol=1e-14, max_iter=5000)
    return 0.5 * np.sum((r.x - xt) ** 2), r.x, A


def test_adjoint_gradient_matches_dense_and_fd():
    c, a, ab, xt = _adjoint_setup()
    L0, x, A = _loss(c, a, ab, xt)
    g = x - xt
    lam = O.pcg(A, g, tol=1e-14, max_iter=5000, transpose=True).x
    D = dense_case(LduCase("t", c.n_cells, c.owner, c.neighbour, A.diag, a, a))
    assert np.linalg.norm(lam - np.linalg.solve(D.T, g)) <= 1e-11 * np.linalg.norm(lam)
    gd, gu, gl = O.coeff_grad(A, lam, x)
    G = -np.outer(lam, x)  # dL/dA_ij = -lambda_i x_j
    assert np.allclose(gd, np.diag(G), rtol=1e-14, atol=0)
    assert np.allclose(gu, G[c.owner, c.neighbour], rtol=1e-14, atol=0)
    assert np.allclose(gl, G[c.neighbour, c.owner], rtol=1e-14, atol=0)
    # symmetric face coefficient c_f: upper = lower = c_f, diag -= c_f at both ends
    gc = gu + gl - gd[c.owner] - gd[c.neighbour]
    closed = (lam[c.owner] - lam[c.neighbour]) * (x[c.owner] - x[c.neighbour])
    assert np.allclose(gc, closed, rtol=1e-10, atol=1e-14 * np.abs(closed).max())
    for f in np.random.default_rng(5).choice(c.n_faces, 8, replace=False):
        h = 1e-6 * a[f]
        ap = a.copy(); ap[f] += h
        am = a.copy(); am[f] -= h
        fd = (_loss(c, ap, ab, xt)[0] - _loss(c, am, ab, xt)[0]) / (2 * h)
        assert abs(fd - gc[f]) <= 1e-5 * max(abs(gc[f]), 1e-3 * np.abs(gc).max())


def test_adjoint_of_symmetric_is_forward():
    c = box_case(5, 4, 4, coeff="lognormal", dirichlet_x0=2.0, seed=30)
    A = O.Ldu.from_case(c)
    f = O.pcg(A, c.rhs[0], tol=1e-12)
    t = O.pcg(A, c.rhs[0], tol=1e-12, transpose=True)
    assert np.array_equal(f.x, t.x)


# ---------------------------------------------------------------- CG + V-cycle

def test_vcycle_pcg_exact_preconditioner_one_iteration():
    """With a single level the V-cycle is the coarsest solve (CG to 1e-10),
    i.e. nearly A^-1, so the preconditioned CG stops after one iteration."""
    c = box_case(4, 3, 3, coeff="lognormal", dirichlet_x0=1.0, seed=40)
    g = O.Gamg(O.Ldu.from_case(c), n_coarsest=1000)
    assert g.n_levels == 1
    r = g.pcg(c.rhs[0], tol=1e-8)
    assert r.status == O.OK and r.iterations == 1


def test_vcycle_pcg_matches_dense_and_beats_diagonal():
    c = _perm_case(box_case(9, 8, 7, coeff="lognormal", sigma=1.0,
                            dirichlet_x0=1.0, seed=41), 42)
    A = O.Ldu.from_case(c)
    g = O.Gamg(A, n_coarsest=10)
    r = g.pcg(c.rhs[0], tol=1e-12)
    xd = np.linalg.solve(dense_case(c), c.rhs[0])
    assert r.status == O.OK
    assert np.linalg.norm(r.x - xd) <= 1e-10 * np.linalg.norm(xd)
    assert r.iterations < O.pcg(A, c.rhs[0], tol=1e-12).iterations / 2


def test_set_values_equals_fresh_galerkin_on_same_aggregation():
    c = box_case(7, 6, 5, coeff="lognormal", dirichlet_x0=1.0, seed=43)
    g = O.Gamg(O.Ldu.from_case(c), n_coarsest=10)
    a2 = c.upper * np.exp(0.3 * np.random.default_rng(44).standard_normal(c.n_faces))
    d2 = assemble_diag(c.n_cells, c.owner, c.neighbour, a2, a2,
                       np.where(np.arange(c.n_cells) % 7 == 0, 1.0, 0.0))
    aggs = [g.level(l).agg for l in range(g.n_levels - 1)]
    g.set_values(d2, a2, a2)
    Af = dense(c.n_cells, c.owner, c.neighbour, d2, a2, a2)
    for l in range(g.n_levels - 1):
        F, Cl = g.level(l), g.level(l + 1)
        assert np.array_equal(F.agg, aggs[l])
        P = prolongation(F.agg, Cl.n)
        Ac = dense(Cl.n, Cl.owner, Cl.neighbour, Cl.diag, Cl.upper, Cl.lower)
        ref = P.T @ Af @ P
        assert np.allclose(Ac, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
        Af = Ac


def test_mixed_vcycle_pcg_refines_to_fp64_solution():
    c = _perm_case(box_case(9, 8, 7, coeff="lognormal", sigma=1.0,
                            dirichlet_x0=1.0, seed=45), 46)
    g = O.Gamg(O.Ldu.from_case(c), n_coarsest=10)
    xd = np.linalg.solve(dense_case(c), c.rhs[0])
    r = g.pcg_mixed(c.rhs[0], tol=1e-12, n_pre=1, n_post=1)
    assert r.status == O.OK and r.true_residual <= 1e-12
    assert np.linalg.norm(r.x - xd) <= 1e-10 * np.linalg.norm(xd)
    assert r.iterations <= 6


# ---------------------------------------------------------------- aggressive agglomeration

@pytest.mark.parametrize("passes", [2, 3])
@pytest.mark.parametrize("idx", range(4))
def test_aggressive_agglomeration_composes_pairwise_passes(idx, passes):
    """passes > 1: pass k pairs the aggregates of pass k-1 on their Galerkin
    matrix; built here from the dense definitions and composed."""
    c = _match_cases()[idx]
    g = O.Gamg(O.Ldu.from_case(c), n_coarsest=2, max_levels=2, match_rounds=100000,
               passes=passes)
    n, own, nb, d, up, lo = c.n_cells, c.owner, c.neighbour, c.diag, c.upper, c.lower
    comp = np.arange(c.n_cells)
    for _ in range(passes):
        agg, nc = pairwise_aggregation(n, own, nb, up, lo, d)
        comp = agg[comp]
        if nc <= 1:
            break
        own, nb, d, up, lo = galerkin_ldu(n, own, nb, d, up, lo, agg, nc)
        n = nc
    assert np.array_equal(g.level(0).agg, comp)
    # and the coarse matrix is P^T A P for the composed aggregation
    C1 = g.level(1)
    ro, rn, rd, ru, rl = galerkin_ldu(c.n_cells, c.owner, c.neighbour, c.diag, c.upper,
                                      c.lower, comp, C1.n)
    assert C1.n == comp.max() + 1
    assert np.array_equal(C1.owner, ro) and np.array_equal(C1.neighbour, rn)
    tol = 1e-14 * np.abs(c.diag).max()
    assert np.allclose(C1.diag, rd, rtol=0, atol=tol)
    assert np.allclose(C1.upper, ru, rtol=0, atol=tol)
    assert np.allclose(C1.lower, rl, rtol=0, atol=tol)


def test_aggressive_agglomeration_fewer_levels_and_converges():
    c = box_case(12, 11, 10, coeff="lognormal", dirichlet_x0=1.0, seed=47)
    A = O.Ldu.from_case(c)
    levels = []
    for passes in (1, 2, 3):
        g = O.Gamg(A, passes=passes)
        levels.append(g.n_levels)
        r = g.solve(c.rhs[0], tol=1e-8, max_cycles=500)
        assert r.status == O.OK
        assert np.linalg.norm(c.rhs[0] - O.amul(A, r.x)) <= 1e-8 * np.linalg.norm(c.rhs[0])
    assert levels[0] > levels[1] > levels[2]


# ---------------------------------------------------------------- two-stage Gauss-Seidel, DIC

def _tri_parts(c):
    D = dense_case(c)
    return D, np.diag(np.diag(D)), np.tril(D, -1), np.triu(D, 1)


def test_gs2_inner_steps_converge_to_the_triangular_solve():
    """D^-1 L is nilpotent, so the inner Jacobi-Richardson steps give
    (D + L)^-1 t exactly once their number reaches the longest chain of the
    lower-triangular graph (n - 1 on a 1D chain), and not before."""
    from scipy.linalg import solve_triangular
    c = box_case(9, 1, 1, coeff="lognormal", dirichlet_x0=1.0, seed=51)
    A = O.Ldu.from_case(c)
    D, Dg, L, U = _tri_parts(c)
    r = np.random.default_rng(52).standard_normal(c.n_cells)
    fwd = solve_triangular(Dg + L, r, lower=True)
    bwd = solve_triangular(Dg + U, r, lower=False)
    n = c.n_cells
    for backward, ref in ((False, fwd), (True, bwd)):
        exact = O.gs2_sweep(A, r, backward=backward, inner=n - 1)
        assert np.linalg.norm(exact - ref) <= 1e-13 * np.linalg.norm(ref)
        short = O.gs2_sweep(A, r, backward=backward, inner=n - 2)
        assert np.linalg.norm(short - ref) > 1e-6 * np.linalg.norm(ref)
    # a sweep from a nonzero e corrects by the triangular solve of r - A e
    e0 = np.random.default_rng(53).standard_normal(n)
    got = O.gs2_sweep(A, r, e0, inner=n - 1)
    want = e0 + solve_triangular(Dg + L, r - D @ e0, lower=True)
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)


def test_gs2_unstructured_limit_and_one_step_bound():
    from scipy.linalg import solve_triangular
    c = _perm_case(box_case(5, 4, 3, coeff="lognormal", nonsym=0.4, dirichlet_x0=1.0,
                            seed=54), 55)
    A = O.Ldu.from_case(c)
    D, Dg, L, U = _tri_parts(c)
    r = np.random.default_rng(56).standard_normal(c.n_cells)
    ref = solve_triangular(Dg + L, r, lower=True)
    got = O.gs2_sweep(A, r, inner=c.n_cells)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    # backward sweeps solve with D + U; the coefficients are nonsymmetric, so
    # taking the lower ones here would be caught
    bref = solve_triangular(Dg + U, r, lower=False)
    bgot = O.gs2_sweep(A, r, backward=True, inner=c.n_cells)
    assert np.linalg.norm(bgot - bref) <= 1e-12 * np.linalg.norm(bref)
    # one inner step: the error of the triangular solve is (D^-1 L)^2 applied
    # to the exact answer, so it is bounded by ||D^-1 L||^2 ||ref||
    one = O.gs2_sweep(A, r, inner=1)
    K = np.linalg.norm(np.linalg.solve(Dg, L), 2)
    assert np.linalg.norm(one - ref) <= K ** 2 * np.linalg.norm(ref) * (1 + 1e-12)


def test_gs2_fp32_sweep_is_the_fp64_sweep_to_fp32_rounding():
    """The mixed-precision smoother: on FP32-representable data, each inner
    step of the FP32 sweep rounds a row sum of at most 7 terms and one
    division, and the steps contract (diagonally dominant rows), so it agrees
    with the FP64 sweep to a few hundred FP32 units; a wrong operand or sign
    moves it by O(1)."""
    c = _perm_case(box_case(6, 5, 4, coeff="lognormal", nonsym=0.4, dirichlet_x0=1.0,
                            seed=57), 58)
    A = O.Ldu.from_case(c)
    A32 = O.Ldu(c.n_cells, c.owner, c.neighbour,
                *(v.astype(np.float32).astype(np.float64) for v in (A.diag, A.upper,
                                                                    A.lower)))
    rng = np.random.default_rng(59)
    r = rng.standard_normal(c.n_cells).astype(np.float32)
    e0 = rng.standard_normal(c.n_cells).astype(np.float32)
    eps = np.finfo(np.float32).eps
    for backward in (False, True):
        for inner in (1, 3):
            for e in (None, e0):
                want = O.gs2_sweep(A32, r.astype(np.float64),
                                   None if e is None else e.astype(np.float64),
                                   backward=backward, inner=inner)
                got = O.gs2_sweep_f32(A32, r, e, backward=backward, inner=inner)
                assert got.dtype == np.float32
                err = np.linalg.norm(got - want) / np.linalg.norm(want)
                assert err <= 300 * eps, (backward, inner, e is None, err)


@pytest.mark.parametrize("smoother", ["jacobi", "gs2"])
def test_fp32_vcycle_is_the_fp64_vcycle_to_fp32_rounding(smoother):
    """The mixed-precision V-cycle is the FP64 V-cycle (pinned to dense
    formulas above) with FP32 arithmetic: on FP32-representable coefficients
    and residual, with the coarsest level solved in FP64 to 1e-10, the two
    agree to FP32 rounding (measured about 1e-7), forward and transposed,
    with and without the correction scaling.  A swapped sweep direction or a
    wrong operand anywhere in the FP32 cycle moves the result by O(1)."""
    c = _perm_case(box_case(7, 6, 5, coeff="lognormal", nonsym=0.4, dirichlet_x0=1.0,
                            seed=61), 62)
    A = O.Ldu.from_case(c)
    A32 = O.Ldu(c.n_cells, c.owner, c.neighbour,
                *(v.astype(np.float32).astype(np.float64) for v in (A.diag, A.upper,
                                                                    A.lower)))
    g = O.Gamg(A32, n_coarsest=4, smoother=smoother, gs_inner=2)
    assert g.n_levels >= 4
    r = np.random.default_rng(63).standard_normal(c.n_cells).astype(np.float32)
    eps = np.finfo(np.float32).eps
    for scale in (False, True):
        for tr in (False, True):
            want = g.vcycle(r.astype(np.float64), n_pre=2, n_post=2, scale=scale,
                            transpose=tr)
            got = g.vcycle_f32(r, n_pre=2, n_post=2, scale=scale, transpose=tr)
            err = np.linalg.norm(got - want) / np.linalg.norm(want)
            assert err <= 100 * eps, (scale, tr, err)


def test_vcycle_gs2_two_level_dense_formula():
    """With exact triangular solves the two-stage smoother is Gauss-Seidel:
    forward sweeps before the coarse correction, backward sweeps after."""
    from scipy.linalg import solve_triangular
    c = box_case(5, 4, 3, coeff="lognormal", dirichlet_x0=1.0, seed=3)
    n = c.n_cells
    g = O.Gamg(O.Ldu.from_case(c), n_coarsest=40, max_levels=2, smoother="gs2",
               gs_inner=n)
    assert g.n_levels == 2
    D, Dg, L, U = _tri_parts(c)
    P = prolongation(g.level(0).agg, g.level(1).n)
    Ac = P.T @ D @ P
    r = np.random.default_rng(57).standard_normal(n)
    e = solve_triangular(Dg + L, r, lower=True)
    e = e + solve_triangular(Dg + L, r - D @ e, lower=True)
    t = r - D @ e
    cc = P @ np.linalg.solve(Ac, P.T @ t)
    e = e + ((cc @ t) / (cc @ (D @ cc))) * cc
    for _ in range(2):
        e = e + solve_triangular(Dg + U, r - D @ e, lower=False)
    got = g.vcycle(r, n_pre=2, n_post=2, scale=True)
    assert np.linalg.norm(got - e) <= 1e-8 * np.linalg.norm(e)


@pytest.mark.parametrize("inner", [1, 2])
def test_vcycle_gs2_is_symmetric_without_scaling(inner):
    c = box_case(7, 6, 5, coeff="lognormal", dirichlet_x0=1.0, seed=9)
    g = O.Gamg(O.Ldu.from_case(c), n_coarsest=10, smoother="gs2", gs_inner=inner)
    rng = np.random.default_rng(58)
    u, v = rng.standard_normal((2, c.n_cells))
    Vu = g.vcycle(u, scale=False)
    Vv = g.vcycle(v, scale=False)
    assert abs(u @ Vv - v @ Vu) <= 1e-8 * np.linalg.norm(u) * np.linalg.norm(Vv)
    # but not with forward sweeps on both sides: the pairing matters
    g2 = O.Gamg(O.Ldu.from_case(c), n_coarsest=10, smoother="gs2", gs_inner=inner)
    Vu1 = g2.vcycle(u, n_pre=1, n_post=0, scale=False)
    Vv1 = g2.vcycle(v, n_pre=1, n_post=0, scale=False)
    assert abs(u @ Vv1 - v @ Vu1) > 1e-6 * np.linalg.norm(u) * np.linalg.norm(Vv1)


@pytest.mark.parametrize("nonsym", [0.0, 0.5])
def test_dic_reproduces_the_diagonal_and_inverts_its_factors(nonsym):
    c = _perm_case(box_case(5, 4, 3, coeff="lognormal", nonsym=nonsym, dirichlet_x0=1.0,
                            seed=59), 60)
    A = O.Ldu.from_case(c)
    D, Dg, L, U = _tri_parts(c)
    r = np.random.default_rng(61).standard_normal(c.n_cells)
    dt, ok, z = O.dic(A, r)
    assert ok
    Dt = np.diag(dt)
    M = (Dt + L) @ np.diag(1.0 / dt) @ (Dt + U)
    # the modified pivots make diag(M) = diag(A); on a box mesh (no
    # triangles in the graph) M - A also vanishes on A's off-diagonal pattern
    assert np.allclose(np.diag(M), np.diag(D), rtol=1e-13, atol=0)
    pat = (D != 0) & ~np.eye(c.n_cells, dtype=bool)
    assert np.max(np.abs((M - D)[pat])) <= 1e-13 * np.abs(D).max()
    assert np.linalg.norm(M @ z - r) <= 1e-13 * np.linalg.norm(r) * np.linalg.cond(M)


def test_dic_is_exact_on_a_chain_and_falls_back_when_singular():
    c = box_case(10, 1, 1, coeff="lognormal", dirichlet_x0=1.0, seed=62)
    A = O.Ldu.from_case(c)
    r = np.random.default_rng(63).standard_normal(c.n_cells)
    _, ok, z = O.dic(A, r)
    # a tridiagonal matrix has no fill: M = A
    assert ok and np.allclose(z, np.linalg.solve(dense_case(c), r), rtol=1e-12, atol=0)
    # pure zero-gradient chain: the last exact pivot is 0, so the level uses
    # the diagonal preconditioner
    cs = box_case(10, 1, 1, coeff="lognormal", seed=64)
    As = O.Ldu.from_case(cs)
    _, oks, zs = O.dic(As, r)
    assert not oks and np.array_equal(zs, r / cs.diag)


@pytest.mark.parametrize("smoother,coarsest", [("gs2", "diag"), ("jacobi", "dic"),
                                               ("gs2", "dic")])
def test_gamg_variants_converge_to_dense_solution(smoother, coarsest):
    c = _perm_case(box_case(8, 7, 6, coeff="lognormal", dirichlet_x0=1.0, seed=12), 13)
    A = O.Ldu.from_case(c)
    xd = np.linalg.solve(dense_case(c), c.rhs[0])
    g = O.Gamg(A, n_coarsest=60, smoother=smoother, coarsest=coarsest)
    r = g.solve(c.rhs[0], tol=1e-12, max_cycles=500)
    assert r.status == O.OK and np.linalg.norm(r.x - xd) <= 1e-10 * np.linalg.norm(xd)
    p = g.pcg(c.rhs[0], tol=1e-12)
    assert p.status == O.OK and np.linalg.norm(p.x - xd) <= 1e-10 * np.linalg.norm(xd)
    # a one-level hierarchy is the coarsest solve itself: 1e-10 relative
    g1 = O.Gamg(A, n_coarsest=10 ** 6, coarsest=coarsest)
    e = g1.vcycle(c.rhs[0])
    assert np.linalg.norm(c.rhs[0] - O.amul(A, e)) <= 1e-10 * np.linalg.norm(c.rhs[0])


def test_aggressive_from_keeps_pairwise_levels_above():
    """aggressive_from = k: levels above k coarsen exactly as plain pairwise
    agglomeration does; level k onwards uses the composed passes."""
    c = box_case(12, 11, 10, coeff="lognormal", dirichlet_x0=1.0, seed=48)
    A = O.Ldu.from_case(c)
    g1 = O.Gamg(A, passes=1)
    for k in (1, 2):
        gk = O.Gamg(A, passes=3, aggressive_from=k)
        for l in range(k):
            assert np.array_equal(gk.level(l).agg, g1.level(l).agg)
        assert gk.level(k).n == g1.level(k).n
        # below: the composed three-pass aggregation of level k's matrix
        Lk = gk.level(k)
        sub = O.Gamg(O.Ldu(Lk.n, Lk.owner, Lk.neighbour, Lk.diag, Lk.upper, Lk.lower),
                     passes=3, max_levels=2, n_coarsest=1)
        assert np.array_equal(gk.level(k).agg, sub.level(0).agg)
        assert gk.n_levels < g1.n_levels


# ---------------------------------------------------------------- PBiCG

@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("precond", [False, True])
def test_pbicg_solves_nonsymmetric_dense(transpose, precond):
    from meshgen import config_case
    for c in (_perm_case(box_case(6, 5, 4, coeff="lognormal", nonsym=0.6, dirichlet_x0=1.0,
                                  seed=71), 72),
              config_case("c5u", n=7)):
        A = O.Ldu.from_case(c)
        D = dense_case(c)
        r = O.pbicg(A, c.rhs[0], tol=1e-12, precond=precond, transpose=transpose)
        xd = np.linalg.solve(D.T if transpose else D, c.rhs[0])
        assert r.status == O.OK and r.true_residual <= 1e-12
        assert np.linalg.norm(r.x - xd) <= 1e-10 * np.linalg.norm(xd)


def test_pbicg_is_cg_on_symmetric_matrices():
    """With A and M symmetric the shadow sequence equals the primal one, so
    BiCG's recurrences are CG's, step for step."""
    c = _perm_case(box_case(8, 7, 6, coeff="lognormal", dirichlet_x0=1.0, seed=73), 74)
    A = O.Ldu.from_case(c)
    for precond in (False, True):
        rb = O.pbicg(A, c.rhs[0], tol=1e-10, precond=precond)
        rc = O.pcg(A, c.rhs[0], tol=1e-10, precond=precond)
        assert rb.iterations == rc.iterations
        assert np.array_equal(rb.history, rc.history)
        assert np.array_equal(rb.x, rc.x)


def test_pbicg_zero_rhs_and_warm_start():
    from meshgen import config_case
    c = config_case("c5u", n=6)
    A = O.Ldu.from_case(c)
    r0 = O.pbicg(A, np.zeros(c.n_cells))
    assert r0.status == O.OK and r0.iterations == 0 and not r0.x.any()
    xd = np.linalg.solve(dense_case(c), c.rhs[0])
    rw = O.pbicg(A, c.rhs[0], x0=xd, tol=1e-8)
    assert rw.status == O.OK and rw.iterations <= 1


# ---------------------------------------------------------------- pressure assembly

def test_assembly_uniform_box_is_the_seven_point_stencil():
    """gamma = 1 on a uniform box with spacing h: every face coefficient is
    |S| / |d| = h, and the matrix is h times the 7-point Laplacian (closed
    form: dense stencil built from cell coordinates)."""
    n = 5
    h = 1.0 / n
    own, nb, ax = box_faces(n, n, n)
    N = n ** 3
    d, u, lo, _ = O.assemble_pressure(N, own, nb, np.ones(N), np.full(own.size, 0.5),
                                      np.full(own.size, h * h), np.full(own.size, 1.0 / h))
    assert np.allclose(u, h, rtol=1e-15) and np.array_equal(u, lo)
    ijk = np.stack(np.unravel_index(np.arange(N), (n, n, n)), 1)
    S = np.zeros((N, N))
    for i in range(N):
        for j in range(N):
            if np.abs(ijk[i] - ijk[j]).sum() == 1:
                S[i, j] = h
    np.fill_diagonal(S, -S.sum(1))
    assert np.allclose(dense(N, own, nb, d, u, lo), S, rtol=0, atol=1e-15)


def test_assembly_column_sums_divergence_and_interpolation():
    g = c3_assembly_inputs(n=12)
    N, own, nb = g["n"], g["owner"], g["neighbour"]
    d, u, lo, b = O.assemble_pressure(N, own, nb, g["gamma"], g["weights"], g["mag_sf"],
                                      g["delta"], g["diag_bc"], g["phi"], g["b_bc"])
    A = dense(N, own, nb, d, u, lo)
    # negSumDiag: each column sums to minus its boundary coefficient
    assert np.allclose(A.sum(0), -g["diag_bc"], rtol=0, atol=1e-13 * np.abs(d).max())
    # divergence telescopes: interior fluxes cancel in the total
    assert abs(b.sum() - g["b_bc"].sum()) <= 1e-14 * np.abs(g["phi"]).sum()
    # the boundary source is added to the divergence cell by cell
    bbc = np.random.default_rng(60).standard_normal(N)
    _, _, _, b2 = O.assemble_pressure(N, own, nb, g["gamma"], g["weights"], g["mag_sf"],
                                      g["delta"], g["diag_bc"], g["phi"], bbc)
    assert np.allclose(b2 - b, bbc - g["b_bc"], rtol=0, atol=1e-14 * np.abs(b).max())
    # a uniform flux through x faces only leaves sources on the x = 0 / x = end layers
    phi_x = np.where(own + 1 == nb, 1.0, 0.0)
    _, _, _, bx = O.assemble_pressure(N, own, nb, g["gamma"], g["weights"], g["mag_sf"],
                                      g["delta"], phi=phi_x)
    m = g["shape"][0]
    ix = np.arange(N) % m
    assert np.all(bx[(ix > 0) & (ix < m - 1)] == 0.0)
    assert np.all(bx[ix == 0] == 1.0) and np.all(bx[ix == m - 1] == -1.0)
    # linear interpolation is exact for a field linear in z (graded spacing)
    dx, dz = c3_spacing(g["shape"][2])
    zc = np.cumsum(dz) - 0.5 * dz
    z = zc[np.arange(N) // (m * m)]
    _, uz, _, _ = O.assemble_pressure(N, own, nb, 1.0 + z, g["weights"],
                                      np.ones(own.size), np.ones(own.size))
    zf = np.where(nb - own == m * m, np.cumsum(dz)[own // (m * m)], z[own])
    assert np.allclose(uz, 1.0 + zf, rtol=1e-14, atol=0)


# ---------------------------------------------------------------- match-round cap

def _sawtooth_chain(blocks=3, length=36, diag=-100.0):
    """A chain of blocks*length cells, faces (i, i+1).  Inside a block the
    coupling grows strictly towards the block's last face; the face joining
    two blocks is the weakest of all.  With a constant diagonal the matching
    weight is a monotone function of the coupling, so a handshake round pairs
    exactly the top free pair of each block: after k rounds each block holds
    min(k, length // 2) pairs, and a cap of k rounds binds for k < length / 2."""
    n = blocks * length
    own = np.arange(n - 1, dtype=np.int32)
    nb = own + 1
    pos = own % length
    a = np.where(pos == length - 1, 0.01, 1.0 + pos.astype(np.float64))
    return n, own, nb, np.full(n, diag), a


@pytest.mark.parametrize("rounds", [1, 2, 16, 17, 100000])
def test_match_round_cap_binds(rounds):
    from dense_ref import handshake_rounds
    n, own, nb, d, a = _sawtooth_chain()
    g = O.Gamg(O.Ldu(n, own, nb, d, a, a), n_coarsest=2, max_levels=2,
               match_rounds=rounds)
    assert g.n_levels == 2
    partner = g.level(0).partner
    ref = handshake_rounds(n, own, nb, a, rounds)
    assert np.array_equal(partner, ref)
    pairs = int(np.sum(partner >= 0)) // 2
    assert pairs == 3 * min(rounds, 18)


# ---------------------------------------------------------------- FP32 inner CG

@pytest.mark.parametrize("steps", [1, 2, 3])
def test_pcg32_inner_steps_bit_exact(steps):
    """One refinement step from x0 = 0 with an inner CG of exactly `steps`
    iterations (no stopping test can fire: outer tolerance 0, inner 1e-300)
    returns x = s * d with s = max|b| and d the FP32 inner iterate."""
    from dense_ref import pcg32_inner_steps
    c = _perm_case(box_case(4, 3, 3, coeff="lognormal", dirichlet_x0=1.0, seed=51), 52)
    A = O.Ldu.from_case(c)
    b = c.rhs[0]
    r = O.pcg_mixed(A, b, tol=0.0, max_refine=1, inner_tol=1e-300,
                    inner_max_iter=steps)
    assert r.status == O.NOT_CONVERGED and r.iterations == 1
    assert r.inner_iterations == steps
    s = np.abs(b).max()
    rhat = (b / s).astype(np.float32)
    dref = pcg32_inner_steps(c.n_cells, c.owner, c.neighbour, c.diag, c.upper, c.lower,
                             rhat, steps)
    assert np.array_equal(r.x, s * dref.astype(np.float64))
