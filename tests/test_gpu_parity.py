"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Bars: integer/addressing results bit-exact; Amul, Tmul, FP32 Amul and the
Galerkin hierarchy bit-exact (same rounding sequence as the oracle's face
loops); FP64 solves: equal iteration counts, residual histories within 1e-9
relative, solutions within 1e-10 relative; the true residual of every GPU
solution is recomputed by the oracle.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
from meshgen import box_case, config_case, random_order, relabel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _lib():
    from paper_2512_22215_amd import LduMatrix
    return LduMatrix


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _perm(c, seed):
    return relabel(c, random_order(c.n_cells, np.random.default_rng(seed)))


def _cases():
    return {
        "c1": config_case("c1"),
        "ragged": _perm(box_case(37, 29, 11, coeff="lognormal", dirichlet_x0=1.0, seed=3), 4),
        "nonsym": _perm(box_case(13, 9, 7, coeff="lognormal", nonsym=0.6, seed=5), 6),
        "tiny": box_case(3, 2, 1, coeff="lognormal", dirichlet_x0=1.0, seed=7),
        "single": box_case(1, 1, 1, coeff="uniform", dirichlet_x0=1.0),
    }


CASES = _cases()


def hist_close(h, ref, rel=1e-9):
    """Residual histories agree to rel, above the FP64 noise floor of a
    recomputed residual ||b - A x|| / ||b|| (about 1e-15 for these systems:
    n-term sums of O(||A|| ||x||) products, rounded at 2^-53)."""
    h = np.asarray(h)
    return h.shape == ref.shape and bool(np.all(np.abs(h - ref) <= rel * ref + 1e-15))


def expected_downleg(g, level, plain):
    """The one-pass down leg the library builds for level `level` of the
    oracle hierarchy g: a plain-slice level above 300,000 coarse rows runs
    over its own scaled slices; otherwise R, in compressed slices above
    300,000 rows, else in CSR with G lanes per row, G the power of two
    nearest (entries per row) / 2, from 1 to 16 (R's entries: the union of
    the members' columns and their diagonals, counted here with scipy)."""
    import scipy.sparse as sp
    L, C = g.level(level), g.level(level + 1)
    if C.n > 300000:
        return ("scaled_slices", 0) if plain else ("r_compressed", 0)
    rows = np.concatenate([L.owner, L.neighbour, np.arange(L.n)])
    cols = np.concatenate([L.neighbour, L.owner, np.arange(L.n)])
    M = sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(L.n, L.n))
    P = sp.csr_matrix((np.ones(L.n), (np.arange(L.n), L.agg)), shape=(L.n, C.n))
    nnz = (P.T @ M).tocsr().nnz
    per = nnz / C.n / 2
    lanes = 1
    while lanes < 16 and 2.0 * lanes <= per * 1.41421356:
        lanes *= 2
    return "r_csr", lanes


def true_res(c, x):
    A = O.Ldu.from_case(c)
    b = c.rhs[0]
    return np.linalg.norm(b - O.amul(A, x)) / np.linalg.norm(b)


@pytest.mark.parametrize("name", list(CASES))
def test_amul_tmul_bit_exact(name):
    c = CASES[name]
    m = _lib().from_case(c)
    A = O.Ldu.from_case(c)
    x = np.random.default_rng(1).standard_normal(c.n_cells)
    y = m.amul(_t(x)).cpu().numpy()
    yt = m.tmul(_t(x)).cpu().numpy()
    assert np.array_equal(y, O.amul(A, x))
    assert np.array_equal(yt, O.tmul(A, x))
    x32 = x.astype(np.float32)
    y32 = m.amul_f32(_t(x32)).cpu().numpy()
    assert np.array_equal(y32, O.amul_f32(A, x32))


@pytest.mark.parametrize("order,side", [("natural", 48), ("mixed", 48), ("random", 48),
                                        ("random", 64)])
def test_column_storage_forms_bit_exact(order, side):
    """Boxes beyond what 16-bit columns can address (48^3 = 110,592 cells,
    64^3 = 262,144).  A slot (the k-th entries of a slice's rows) that spans
    at most 65535 columns is read as 16-bit offsets from its smallest column,
    a wider one as 32-bit columns.  Natural numbering: every slot narrow.
    The first 30% of the cells in order and the rest shuffled: both kinds in
    one level (about 5% wide), as in random numbering at 48^3 (about 77%
    wide).  Random numbering at 64^3: every slot wide, no 16-bit array.  All
    give the oracle's Amul, Tmul and FP32 Amul bit for bit, and the same GAMG
    solve."""
    c = box_case(side, side, side, coeff="lognormal", nonsym=0.3, dirichlet_x0=1.0, seed=31)
    if order == "random":
        c = _perm(c, 32)
    elif order == "mixed":
        n0 = int(0.3 * c.n_cells)
        tail = n0 + np.random.default_rng(34).permutation(c.n_cells - n0)
        c = relabel(c, np.concatenate([np.arange(n0), tail]))
    m = _lib().from_case(c)
    lay = m.layout(0)
    assert lay == {"compressed": False, "col16": not (order == "random" and side == 64)}
    A = O.Ldu.from_case(c)
    x = np.random.default_rng(33).standard_normal(c.n_cells)
    assert np.array_equal(m.amul(_t(x)).cpu().numpy(), O.amul(A, x))
    assert np.array_equal(m.tmul(_t(x)).cpu().numpy(), O.tmul(A, x))
    x32 = x.astype(np.float32)
    assert np.array_equal(m.amul_f32(_t(x32)).cpu().numpy(), O.amul_f32(A, x32))
    # the coarse levels keep 32-bit columns in compressed slices
    m.gamg_setup(n_pre=1, n_post=1)
    assert m.layout(1) == {"compressed": True, "col16": False}
    b = c.rhs[0]
    xg, sg = m.gamg(_t(b), rel_tol=1e-8, n_pre=1, n_post=1)
    rg = O.Gamg(A).solve(b, tol=1e-8, n_pre=1, n_post=1)
    assert sg.converged and rg.status == O.OK and sg.iterations == rg.iterations
    assert np.linalg.norm(xg.cpu().numpy() - rg.x) <= 1e-10 * np.linalg.norm(rg.x)
    m.close()


def test_create_rejects_bad_input():
    from paper_2512_22215_amd import LduError
    c = CASES["tiny"]
    LduMatrix = _lib()
    bad = c.neighbour.copy()
    bad[0] = c.owner[0]
    with pytest.raises(LduError) as e:
        LduMatrix(c.n_cells, c.owner, bad, c.diag, c.upper, c.lower)
    assert e.value.code == -2
    unsorted = np.ascontiguousarray(c.owner[::-1]), np.ascontiguousarray(c.neighbour[::-1])
    with pytest.raises(LduError) as e:
        LduMatrix(c.n_cells, unsorted[0], unsorted[1], c.diag, c.upper, c.lower)
    assert e.value.code == -2
    d = c.diag.copy()
    d[1] = np.nan
    with pytest.raises(LduError) as e:
        LduMatrix(c.n_cells, c.owner, c.neighbour, d, c.upper, c.lower)
    assert e.value.code == -3


def test_pcg_c1_matches_oracle_and_golden():
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "oracle_c1.json")))
    c = CASES["c1"]
    m = _lib().from_case(c)
    x, st = m.pcg(_t(c.rhs[0]), rel_tol=1e-8, history=1000)
    ref = O.pcg(O.Ldu.from_case(c), c.rhs[0], tol=1e-8)
    xg = x.cpu().numpy()
    assert st.converged and st.iterations == ref.iterations == gold["pcg"]["iterations"]
    assert hist_close(st.history, ref.history)
    assert true_res(c, xg) <= 1e-8
    assert np.linalg.norm(xg - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
    p = c.meta["p_exact"]
    assert np.linalg.norm(xg - p) <= 5e-5 * np.linalg.norm(p)


@pytest.mark.parametrize("name", ["ragged", "tiny", "single"])
def test_pcg_matches_oracle(name):
    c = CASES[name]
    m = _lib().from_case(c)
    x, st = m.pcg(_t(c.rhs[0]), rel_tol=1e-10, history=5000)
    ref = O.pcg(O.Ldu.from_case(c), c.rhs[0], tol=1e-10)
    xg = x.cpu().numpy()
    assert st.converged and st.iterations == ref.iterations
    assert np.linalg.norm(xg - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
    assert true_res(c, xg) <= 1e-10


def test_pcg_edge_cases():
    c = CASES["ragged"]
    m = _lib().from_case(c)
    x, st = m.pcg(torch.zeros(c.n_cells, dtype=torch.float64, device="cuda"),
                  x0=torch.ones(c.n_cells, dtype=torch.float64, device="cuda"))
    assert st.status == 0 and st.iterations == 0 and float(x.abs().max()) == 0.0
    x, st = m.pcg(_t(c.rhs[0]), max_iter=1)
    assert st.status == 1 and st.iterations == 1 and not st.converged
    ref = O.pcg(O.Ldu.from_case(c), c.rhs[0], max_iter=1)
    assert np.linalg.norm(x.cpu().numpy() - ref.x) <= 1e-12 * np.linalg.norm(ref.x)


@pytest.mark.parametrize("k", [1, 2, 15, 16, 17, 33])
def test_iteration_cap_keeps_the_last_update(k):
    """A solve stopped by its iteration cap, inside or at the end of a
    16-iteration check block, has applied its last iteration's x += alpha p,
    which the CG loops defer to the direction update: after k iterations x
    equals the oracle's, for diagonal PCG and for CG + V-cycle (one sweep,
    three matching passes below level 1), forward and transposed (the matrix
    is symmetric, so both match the oracle's forward solve)."""
    c = _gamg_case("c3s")
    A = O.Ldu.from_case(c)
    b = c.rhs[0]
    m = _lib().from_case(c)
    x, st = m.pcg(_t(b), rel_tol=1e-14, max_iter=k)
    ref = O.pcg(A, b, tol=1e-14, max_iter=k)
    print(f"k={k} diag: it {st.iterations} status {st.status}", flush=True)
    assert st.iterations == k == ref.iterations and st.status == 1
    assert np.linalg.norm(x.cpu().numpy() - ref.x) <= 1e-12 * np.linalg.norm(ref.x)
    hier = dict(passes=3, aggressive_from=1)
    m.gamg_setup(n_pre=1, n_post=1, **hier)
    rp = O.Gamg(A, **hier).pcg(b, tol=1e-14, max_iter=k, n_pre=1, n_post=1)
    for name, (xp, sp) in (("forward", m.pcg(_t(b), precond=2, rel_tol=1e-14, max_iter=k)),
                           ("transposed", m.adjoint(_t(b), solver="pcg", precond=2,
                                                    rel_tol=1e-14, max_iter=k))):
        print(f"k={k} cg+vcycle {name}: it {sp.iterations} status {sp.status}", flush=True)
        assert sp.iterations == k == rp.iterations and sp.status == 1, name
        assert np.linalg.norm(xp.cpu().numpy() - rp.x) <= 1e-10 * np.linalg.norm(rp.x), name
    m.close()


def test_warm_start_matches_oracle():
    """Solvers started from a seeded nonzero x0 (the time loop's warm start):
    iteration counts equal the oracle's from the same x0, and the solutions
    agree: diagonal PCG and CG + V-cycle to 1e-8, the transposed CG + V-cycle
    (the matrix is symmetric), 30 cycles of standalone GAMG, and the mixed
    form refined to 1e-12 against the FP64 oracle."""
    c = _gamg_case("c3s")
    A = O.Ldu.from_case(c)
    b = c.rhs[0]
    x0 = np.random.default_rng(77).standard_normal(c.n_cells)
    m = _lib().from_case(c)
    hier = dict(passes=3, aggressive_from=1)
    m.gamg_setup(n_pre=1, n_post=1, **hier)
    g = O.Gamg(A, **hier)
    runs = [
        ("pcg", m.pcg(_t(b), x0=_t(x0), rel_tol=1e-8), O.pcg(A, b, x0=x0, tol=1e-8), 1e-9),
        ("pcg+vcycle", m.pcg(_t(b), x0=_t(x0), precond=2, rel_tol=1e-8),
         g.pcg(b, x0=x0, tol=1e-8, n_pre=1, n_post=1), 1e-9),
        ("adjoint pcg+vcycle", m.adjoint(_t(b), x0=_t(x0), solver="pcg", precond=2,
                                         rel_tol=1e-8),
         g.pcg(b, x0=x0, tol=1e-8, n_pre=1, n_post=1), 1e-9),
        # standalone GAMG converges slowly on this graded box: 30 cycles
        ("gamg", m.gamg(_t(b), x0=_t(x0), rel_tol=1e-14, n_pre=1, n_post=1, max_cycles=30,
                        **hier),
         g.solve(b, x0=x0, tol=1e-14, n_pre=1, n_post=1, max_cycles=30), 1e-10),
    ]
    for name, (x, st), ref, tol in runs:
        print(f"{name}: it {st.iterations} oracle {ref.iterations} "
              f"residual {st.final_residual:.3e}", flush=True)
        assert st.iterations == ref.iterations, name
        assert st.converged == (ref.status == 0), name
        xr = ref.x
        assert np.linalg.norm(x.cpu().numpy() - xr) <= tol * np.linalg.norm(xr), name
    # the mixed form from the same x0, refined to 1e-12, against the FP64 oracle
    xm, sm = m.pcg(_t(b), x0=_t(x0), precond=2, rel_tol=1e-12, precision="mixed")
    rf = g.pcg(b, x0=x0, tol=1e-12, n_pre=1, n_post=1)
    print(f"mixed: refinements {sm.refinements} inner {sm.iterations}", flush=True)
    assert sm.converged and true_res(c, xm.cpu().numpy()) <= 1e-12
    err = np.linalg.norm(xm.cpu().numpy() - rf.x) / np.linalg.norm(rf.x)
    print(f"mixed vs FP64 oracle: {err:.2e}", flush=True)
    assert err <= 1e-10
    m.close()


def _gamg_case(name):
    if name == "c2s":
        return config_case("c2", n=24)
    if name == "c3p":
        return config_case("c3", nxy=24)  # the 200-layer graded column, 24 x 24 wide
    if name == "c5s":
        return config_case("c5", n=36)
    if name == "c3s":
        # the graded, jittered workload at 40^3
        from meshgen.boxes import _rng, assemble_diag, box_faces, LduCase
        n = 40
        dx = 1.0 / n
        dz = np.minimum((dx / 100.0) * 1.05 ** np.arange(n), dx)
        own, nb, ax = box_faces(n, n, n)
        kz = own // (n * n)
        a = np.where(ax < 2, dz[kz], dx * dx / (0.5 * (dz[kz] + dz[np.minimum(kz + 1, n - 1)])))
        a = a * _rng(3, 2).uniform(0.95, 1.05, own.size)
        ab = np.zeros(n ** 3)
        ab[np.arange(n ** 3) // (n * n) == n - 1] = dx * dx / (0.5 * dz[n - 1])
        d = assemble_diag(n ** 3, own, nb, a, a, ab)
        return LduCase("c3s", n ** 3, own, nb, d, a, a.copy(),
                       [_rng(3, 3).standard_normal(n ** 3)], False)
    return CASES[name]


@pytest.mark.parametrize("name,passes,afrom", [
    ("c2s", 1, 0), ("c3s", 1, 0), ("ragged", 1, 0), ("c1", 1, 0), ("nonsym", 1, 0),
    ("c2s", 2, 0), ("c3s", 2, 0), ("ragged", 3, 0), ("nonsym", 2, 0), ("c3s", 3, 1),
    ("c2s", 3, 2)])
def test_gamg_hierarchy_bit_exact(name, passes, afrom):
    c = _gamg_case(name)
    m = _lib().from_case(c)
    m.gamg_setup(passes=passes, aggressive_from=afrom)
    g = O.Gamg(O.Ldu.from_case(c), passes=passes, aggressive_from=afrom)
    assert m.n_levels() == g.n_levels
    for l in range(g.n_levels):
        got = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in m.level(l).items()}
        ref = g.level(l)
        assert got["n"] == ref.n and got["nf"] == ref.nf
        if ref.agg is not None:
            assert np.array_equal(got["agg"], ref.agg)
        for k, rv in (("owner", ref.owner), ("neighbour", ref.neighbour), ("diag", ref.diag),
                      ("upper", ref.upper), ("lower", ref.lower)):
            assert np.array_equal(got[k], rv), (l, k)


@pytest.mark.parametrize("name", ["c2s", "c3s", "ragged"])
def test_vcycle_matches_oracle(name):
    c = _gamg_case(name)
    m = _lib().from_case(c)
    g = O.Gamg(O.Ldu.from_case(c))
    r = np.random.default_rng(9).standard_normal(c.n_cells)
    if c.singular:
        r -= r.mean()
    e = m.vcycle(_t(r)).cpu().numpy()
    ref = g.vcycle(r)
    assert np.linalg.norm(e - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("name", ["c2s", "c5s", "ragged"])
def test_gamg_solve_matches_oracle(name):
    c = _gamg_case(name)
    m = _lib().from_case(c)
    x, st = m.gamg(_t(c.rhs[0]), rel_tol=1e-8, history=300)
    ref = O.Gamg(O.Ldu.from_case(c)).solve(c.rhs[0], tol=1e-8)
    xg = x.cpu().numpy()
    assert st.converged and st.iterations == ref.iterations
    assert hist_close(st.history, ref.history)
    if c.singular:
        xg = xg - xg.mean()
        xr = ref.x - ref.x.mean()
    else:
        xr = ref.x
    assert np.linalg.norm(xg - xr) <= 1e-10 * np.linalg.norm(xr)
    assert true_res(c, x.cpu().numpy()) <= 1e-8


@pytest.mark.parametrize("passes", [2, 3])
def test_aggressive_agglomeration_solves_match_oracle(passes):
    c = _gamg_case("c5s")
    A = O.Ldu.from_case(c)
    g = O.Gamg(A, passes=passes)
    m = _lib().from_case(c)
    x, st = m.gamg(_t(c.rhs[0]), rel_tol=1e-8, passes=passes, history=300)
    ref = g.solve(c.rhs[0], tol=1e-8)
    assert st.n_levels == g.n_levels and st.converged and st.iterations == ref.iterations
    assert hist_close(st.history, ref.history)
    assert np.linalg.norm(x.cpu().numpy() - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
    # CG preconditioned by the V-cycle of the same hierarchy
    c3 = _gamg_case("c3p")
    A3 = O.Ldu.from_case(c3)
    m3 = _lib().from_case(c3)
    m3.gamg_setup(passes=passes, n_pre=1, n_post=1)
    x3, s3 = m3.pcg(_t(c3.rhs[0]), precond=2, rel_tol=1e-8)
    r3 = O.Gamg(A3, passes=passes).pcg(c3.rhs[0], tol=1e-8, n_pre=1, n_post=1)
    assert s3.converged and s3.iterations == r3.iterations
    assert true_res(c3, x3.cpu().numpy()) <= 1e-8
    assert np.linalg.norm(x3.cpu().numpy() - r3.x) <= 1e-9 * np.linalg.norm(r3.x)


CYCLES = [("gs2", 1, "diag"), ("gs2", 2, "diag"), ("gs2", 3, "dic"), ("jacobi", 1, "dic")]


@pytest.mark.parametrize("smoother,inner,coarsest", CYCLES)
def test_cycle_variants_match_oracle(smoother, inner, coarsest):
    """Two-stage Gauss-Seidel smoothing and the DIC coarsest preconditioner:
    one V-cycle, the GAMG solve and CG + V-cycle against the oracle."""
    kw = dict(smoother=smoother, gs_inner=inner, coarsest=coarsest)
    c = _gamg_case("c5s")
    A = O.Ldu.from_case(c)
    g = O.Gamg(A, **kw)
    m = _lib().from_case(c)
    r = np.random.default_rng(9).standard_normal(c.n_cells)
    e = m.vcycle(_t(r), **kw).cpu().numpy()
    ref = g.vcycle(r)
    assert np.linalg.norm(e - ref) <= 1e-11 * np.linalg.norm(ref)
    x, st = m.gamg(_t(c.rhs[0]), rel_tol=1e-8, history=300, **kw)
    rs = g.solve(c.rhs[0], tol=1e-8)
    assert st.converged and st.iterations == rs.iterations
    assert hist_close(st.history, rs.history)
    assert np.linalg.norm(x.cpu().numpy() - rs.x) <= 1e-10 * np.linalg.norm(rs.x)
    m.gamg_setup(n_pre=1, n_post=1, **kw)
    xp, sp = m.pcg(_t(c.rhs[0]), precond=2, rel_tol=1e-8)
    rp = g.pcg(c.rhs[0], tol=1e-8, n_pre=1, n_post=1)
    assert sp.converged and sp.iterations == rp.iterations
    assert np.linalg.norm(xp.cpu().numpy() - rp.x) <= 1e-9 * np.linalg.norm(rp.x)
    # mixed: FP32 V-cycles with the same smoother, refined to 1e-12
    xm, sm = m.gamg(_t(c.rhs[0]), rel_tol=1e-12, precision="mixed", **kw)
    assert sm.converged and true_res(c, xm.cpu().numpy()) <= 1e-12


def test_coarsest_rows_longer_than_the_register_batch():
    """A 58-cell coarsest level whose longest rows hold 18 entries: the
    one-wavefront coarsest CG takes a row's first 16 entries from registers
    and the rest from LDS.  One V-cycle, the GAMG solve, CG + V-cycle and the
    mixed solve against the oracle."""
    c = _gamg_case("c5s")
    A = O.Ldu.from_case(c)
    g = O.Gamg(A, n_coarsest=64)
    L = g.level(g.n_levels - 1)
    deg = np.bincount(L.owner, minlength=L.n) + np.bincount(L.neighbour, minlength=L.n)
    # one wavefront (at most 64 cells, rows of at most 48 entries), past the batch
    assert L.n <= 64 and 16 < deg.max() <= 48
    b = c.rhs[0]
    m = _lib().from_case(c)
    m.gamg_setup(n_coarsest=64)
    r = np.random.default_rng(9).standard_normal(c.n_cells)
    e = m.vcycle(_t(r), n_coarsest=64).cpu().numpy()
    ref = g.vcycle(r)
    assert np.linalg.norm(e - ref) <= 1e-11 * np.linalg.norm(ref)
    x, st = m.gamg(_t(b), rel_tol=1e-8, n_coarsest=64, history=300)
    rs = g.solve(b, tol=1e-8)
    assert st.n_levels == g.n_levels and st.converged and st.iterations == rs.iterations
    assert hist_close(st.history, rs.history)
    assert np.linalg.norm(x.cpu().numpy() - rs.x) <= 1e-10 * np.linalg.norm(rs.x)
    m.gamg_setup(n_coarsest=64, n_pre=1, n_post=1)
    xp, sp = m.pcg(_t(b), precond=2, rel_tol=1e-8)
    rp = g.pcg(b, tol=1e-8, n_pre=1, n_post=1)
    assert sp.converged and sp.iterations == rp.iterations
    assert np.linalg.norm(xp.cpu().numpy() - rp.x) <= 1e-9 * np.linalg.norm(rp.x)
    # mixed: FP32 V-cycles (FP64 coarsest) refined to 1e-12
    xm, sm = m.gamg(_t(b), rel_tol=1e-12, precision="mixed", n_coarsest=64)
    r12 = g.solve(b, tol=1e-12)
    assert sm.converged and true_res(c, xm.cpu().numpy()) <= 1e-12
    assert np.linalg.norm(xm.cpu().numpy() - r12.x) <= 1e-10 * np.linalg.norm(r12.x)


def test_dic_on_a_large_coarsest_level_and_singular_fallback():
    """A coarsest level too large for the one-wavefront kernel takes the
    workgroup kernel's serial substitution; a singular coarsest level (pure
    zero gradient) may lose its last pivot and then falls back to the
    diagonal, as the oracle does."""
    for name, ncoarse in (("c5s", 400), ("c2s", 50)):
        c = _gamg_case(name)
        A = O.Ldu.from_case(c)
        g = O.Gamg(A, n_coarsest=ncoarse, coarsest="dic")
        m = _lib().from_case(c)
        x, st = m.gamg(_t(c.rhs[0]), rel_tol=1e-8, n_coarsest=ncoarse, coarsest="dic",
                       history=300)
        rs = g.solve(c.rhs[0], tol=1e-8)
        assert st.n_levels == g.n_levels
        assert st.converged and st.iterations == rs.iterations, name
        assert hist_close(st.history, rs.history)
        xg, xr = x.cpu().numpy(), rs.x
        if c.singular:
            xg, xr = xg - xg.mean(), xr - xr.mean()
        assert np.linalg.norm(xg - xr) <= 1e-10 * np.linalg.norm(xr)


@pytest.mark.parametrize("solver", ["pcg", "gamg", "pcg_gamg"])
def test_mixed_refines_to_fp64(solver):
    c = _gamg_case("c5s") if solver == "gamg" else CASES["ragged"]
    if solver == "pcg_gamg":
        c = _gamg_case("c3p")
    m = _lib().from_case(c)
    A = O.Ldu.from_case(c)
    if solver == "pcg":
        x, st = m.pcg(_t(c.rhs[0]), rel_tol=1e-12, precision="mixed")
        ref = O.pcg(A, c.rhs[0], tol=1e-12)
    elif solver == "pcg_gamg":
        x, st = m.pcg(_t(c.rhs[0]), rel_tol=1e-12, precision="mixed", precond=2)
        ref = O.pcg(A, c.rhs[0], tol=1e-12, max_iter=20000)
        orc = O.Gamg(A).pcg_mixed(c.rhs[0], tol=1e-12)
        assert st.refinements == orc.iterations
    else:
        x, st = m.gamg(_t(c.rhs[0]), rel_tol=1e-12, precision="mixed")
        ref = O.Gamg(A).solve(c.rhs[0], tol=1e-12)
    xg = x.cpu().numpy()
    assert st.converged and true_res(c, xg) <= 1e-12
    assert np.linalg.norm(xg - ref.x) <= 1e-10 * np.linalg.norm(ref.x)


def test_adjoint_and_gradients_match_oracle():
    c = CASES["nonsym"]
    m = _lib().from_case(c)
    A = O.Ldu.from_case(c)
    g = np.random.default_rng(3).standard_normal(c.n_cells)
    lam, st = m.adjoint(_t(g), use_gamg=True, rel_tol=1e-12)
    gg = O.Gamg(A)
    ref = gg.solve(g, tol=1e-12, transpose=True)
    assert st.converged and st.iterations == ref.iterations
    lg = lam.cpu().numpy()
    assert np.linalg.norm(lg - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
    x = np.random.default_rng(4).standard_normal(c.n_cells)
    gd, gu, gl = (t.cpu().numpy() for t in m.coeff_grad(lam, _t(x)))
    rd, ru, rl = O.coeff_grad(A, lg, x)
    assert np.array_equal(gd, rd) and np.array_equal(gu, ru) and np.array_equal(gl, rl)


def test_deterministic_bitwise():
    c = _gamg_case("c2s")
    m = _lib().from_case(c)
    x1, _ = m.gamg(_t(c.rhs[0]))
    x2, _ = m.gamg(_t(c.rhs[0]))
    m2 = _lib().from_case(c)
    x3, _ = m2.gamg(_t(c.rhs[0]))
    assert torch.equal(x1, x2) and torch.equal(x1, x3)
    p1, _ = m.pcg(_t(c.rhs[0]))
    p2, _ = m2.pcg(_t(c.rhs[0]))
    assert torch.equal(p1, p2)


def test_interleaved_handles_and_a_side_stream():
    """Two matrices of different sizes, each with its own hierarchy, solved in
    alternation (CG + V-cycle in FP64 and mixed, the adjoint), give bitwise
    the results each gives alone; so does a solve on a side stream (the
    binding passes torch's current stream), and closing one handle leaves
    the other working."""
    ca, cb = _gamg_case("c3s"), CASES["ragged"]
    hier = dict(n_pre=1, n_post=1, passes=3, aggressive_from=1)

    def runs(m, c):
        b = _t(c.rhs[0])
        return [m.pcg(b, precond=2, rel_tol=1e-8)[0],
                m.pcg(b, precond=2, rel_tol=1e-10, precision="mixed")[0],
                m.adjoint(b, solver="pcg", precond=2, rel_tol=1e-8)[0]]

    ma = _lib().from_case(ca)
    ma.gamg_setup(**hier)
    alone_a = runs(ma, ca)
    ma.close()
    mb = _lib().from_case(cb)
    mb.gamg_setup(**hier)
    alone_b = runs(mb, cb)
    mb.close()
    ma, mb = _lib().from_case(ca), _lib().from_case(cb)
    ma.gamg_setup(**hier)
    mb.gamg_setup(**hier)
    ba, bb = _t(ca.rhs[0]), _t(cb.rhs[0])
    got_a, got_b = [], []
    for k, (fa, fb) in enumerate(((lambda: ma.pcg(ba, precond=2, rel_tol=1e-8),
                                   lambda: mb.pcg(bb, precond=2, rel_tol=1e-8)),
                                  (lambda: ma.pcg(ba, precond=2, rel_tol=1e-10, precision="mixed"),
                                   lambda: mb.pcg(bb, precond=2, rel_tol=1e-10, precision="mixed")),
                                  (lambda: ma.adjoint(ba, solver="pcg", precond=2, rel_tol=1e-8),
                                   lambda: mb.adjoint(bb, solver="pcg", precond=2, rel_tol=1e-8)))):
        got_a.append(fa()[0])
        got_b.append(fb()[0])
    for k in range(3):
        assert torch.equal(got_a[k], alone_a[k]) and torch.equal(got_b[k], alone_b[k]), k
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        xs = mb.pcg(bb, precond=2, rel_tol=1e-8)[0]
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    assert torch.equal(xs, alone_b[0])
    ma.close()
    assert torch.equal(mb.pcg(bb, precond=2, rel_tol=1e-8)[0], alone_b[0])
    mb.close()


@pytest.mark.parametrize("name", ["c3p", "c2s", "ragged"])
def test_pcg_gamg_matches_oracle(name):
    c = _gamg_case(name)
    m = _lib().from_case(c)
    x, st = m.pcg(_t(c.rhs[0]), precond=2, rel_tol=1e-8, history=500)
    ref = O.Gamg(O.Ldu.from_case(c)).pcg(c.rhs[0], tol=1e-8)
    xg = x.cpu().numpy()
    assert st.converged and st.iterations == ref.iterations
    assert hist_close(st.history, ref.history, 1e-8)
    if c.singular:
        xg, xr = xg - xg.mean(), ref.x - ref.x.mean()
    else:
        xr = ref.x
    assert np.linalg.norm(xg - xr) <= 1e-9 * np.linalg.norm(xr)
    assert true_res(c, x.cpu().numpy()) <= 1e-8


ONE_SWEEP = dict(n_pre=1, n_post=1, scale_correction=0)


# meshes whose restriction operators have short to long rows, so the CSR
# product runs with 2, 4, 8 and 16 lanes per row (the power of two nearest
# the mean row length over two entries per lane): a chain (rows of about 4
# entries), a plane (about 8), a box (about 13) and a box with three matching
# passes per level below level 1 (about 50)
R_LANE_CASES = {
    "chain": (dict(nx=3000, ny=1, nz=1), {}),
    "plane": (dict(nx=70, ny=60, nz=1), {}),
    "box": (dict(nx=22, ny=20, nz=18), {}),
    "box_aggressive": (dict(nx=22, ny=20, nz=18), dict(passes=3, aggressive_from=1)),
}


@pytest.mark.parametrize("name", list(R_LANE_CASES))
def test_csr_restriction_lane_groups(name):
    """The one-pass down leg through R in CSR, for row lengths that select
    different numbers of lanes per row: CG + V-cycle (FP64, forward and
    transposed) against the oracle's two-step cycle, and the mixed form
    refined to 1e-10."""
    dims, hier = R_LANE_CASES[name]
    c = box_case(dims["nx"], dims["ny"], dims["nz"], coeff="lognormal", dirichlet_x0=1.0,
                 seed=13)
    A = O.Ldu.from_case(c)
    m = _lib().from_case(c)
    m.gamg_setup(**ONE_SWEEP, **hier)
    g = O.Gamg(A, **hier)
    assert m.n_levels() == g.n_levels
    b = c.rhs[0]
    x, st = m.pcg(_t(b), precond=2, rel_tol=1e-8, history=1000)
    ref = g.pcg(b, tol=1e-8, n_pre=1, n_post=1)
    assert st.converged and st.iterations == ref.iterations
    assert hist_close(st.history, ref.history, 1e-8)
    assert np.linalg.norm(x.cpu().numpy() - ref.x) <= 1e-9 * np.linalg.norm(ref.x)
    # the forms the solve ran: R in CSR on every level, with the lanes per row
    # the library's rule gives (over the four cases: 2, 4, 8 and 16)
    forms = [m.downleg(lev) for lev in range(g.n_levels - 1)]
    print(name, forms)
    for lev, f in enumerate(forms):
        assert f == expected_downleg(g, lev, m.layout(lev)["compressed"] is False), (lev, f)
    xt, stt = m.adjoint(_t(b), solver="pcg", precond=2, rel_tol=1e-8)
    reft = g.pcg(b, tol=1e-8, n_pre=1, n_post=1, transpose=True)
    assert stt.converged and stt.iterations == reft.iterations
    # the FP32 cycle (R's values in FP32) inside FP64 refinement, to 1e-10:
    # the chain's condition number is 6.7e7, and its FP64 residual stalls
    # near 6e-12, so 1e-12 is out of reach there in FP64 arithmetic
    xm, sm = m.pcg(_t(b), precond=2, rel_tol=1e-10, precision="mixed")
    assert sm.converged and true_res(c, xm.cpu().numpy()) <= 1e-10
    m.close()


@pytest.mark.parametrize("hier", [{}, dict(passes=3, aggressive_from=1)],
                         ids=["pairwise", "aggressive"])
def test_scaled_slice_down_leg(hier):
    """A plain-slice level with more than 300,000 coarse rows takes its down
    leg over its own slices, t = (I - w A D^-1) r with the values -w a_ij / D_j
    (16-bit columns included), then the member sums of t.  On a 720,000-cell
    box (level 1: about 330,000 cells) against the oracle's two-step cycle:
    V-cycles at two values of w (the second recomputes the values), CG +
    V-cycle forward and transposed, the mixed form to 1e-10, and a V-cycle
    after new coefficients."""
    from meshgen import assemble_diag
    c = box_case(100, 90, 80, coeff="lognormal", dirichlet_x0=1.0, seed=17)
    A = O.Ldu.from_case(c)
    m = _lib().from_case(c)
    m.gamg_setup(**ONE_SWEEP, **hier)
    g = O.Gamg(A, **hier)
    assert m.n_levels() == g.n_levels
    # the case takes the scaled-slice path: plain slices on level 0, a coarse
    # level above the 300,000 rows up to which R is stored in CSR
    assert m.layout(0)["compressed"] is False and m.layout(0)["col16"] is True
    assert g.level(1).n > 300000
    assert m.downleg(0) == ("scaled_slices", 0)
    for lev in range(1, g.n_levels - 1):
        assert m.downleg(lev) == expected_downleg(g, lev, m.layout(lev)["compressed"] is False)
    r = np.random.default_rng(43).standard_normal(c.n_cells)
    # (the agglomeration settings go with every call: a call whose settings
    # differ from the cached hierarchy's builds a new one)
    for omega in (0.75, 0.6, 0.75):
        e = m.vcycle(_t(r), omega=omega, **ONE_SWEEP, **hier).cpu().numpy()
        ref = g.vcycle(r, n_pre=1, n_post=1, omega=omega, scale=False)
        assert np.linalg.norm(e - ref) <= 1e-11 * np.linalg.norm(ref), omega
    b = c.rhs[0]
    m.gamg_setup(**ONE_SWEEP, **hier)
    x, st = m.pcg(_t(b), precond=2, rel_tol=1e-8, history=500)
    ref = g.pcg(b, tol=1e-8, n_pre=1, n_post=1)
    assert st.converged and st.iterations == ref.iterations
    assert hist_close(st.history, ref.history, 1e-8)
    assert np.linalg.norm(x.cpu().numpy() - ref.x) <= 1e-9 * np.linalg.norm(ref.x)
    xt, stt = m.adjoint(_t(b), solver="pcg", precond=2, rel_tol=1e-8)
    reft = g.pcg(b, tol=1e-8, n_pre=1, n_post=1, transpose=True)
    assert stt.converged and stt.iterations == reft.iterations
    assert np.linalg.norm(xt.cpu().numpy() - reft.x) <= 1e-9 * np.linalg.norm(reft.x)
    xm, sm = m.pcg(_t(b), precond=2, rel_tol=1e-10, precision="mixed")
    assert sm.converged and true_res(c, xm.cpu().numpy()) <= 1e-10
    # new face coefficients, the Dirichlet part of the diagonal kept
    a_bc = assemble_diag(c.n_cells, c.owner, c.neighbour, c.upper, c.lower) - c.diag
    a2 = c.upper * np.exp(0.3 * np.random.default_rng(44).standard_normal(c.n_faces))
    d2 = assemble_diag(c.n_cells, c.owner, c.neighbour, a2, a2, a_bc)
    m.set_coeffs(_t(d2), _t(a2), _t(a2))
    g.set_values(d2, a2, a2)
    e = m.vcycle(_t(r), **ONE_SWEEP, **hier).cpu().numpy()
    ref = g.vcycle(r, n_pre=1, n_post=1, scale=False)
    assert np.linalg.norm(e - ref) <= 1e-11 * np.linalg.norm(ref)
    m.close()


@pytest.mark.parametrize("hier", [{}, dict(passes=3, aggressive_from=1)],
                         ids=["pairwise", "aggressive"])
def test_scaled_slice_down_leg_nonsymmetric(hier):
    """The scaled-slice down leg on a non-symmetric 720,000-cell box, where
    the values for A and for A^T differ: a V-cycle and standalone GAMG
    (forward, and on A^T through the adjoint solve) against the oracle."""
    c = box_case(100, 90, 80, coeff="lognormal", nonsym=0.6, dirichlet_x0=1.0, seed=19)
    assert not np.array_equal(c.upper, c.lower)
    A = O.Ldu.from_case(c)
    m = _lib().from_case(c)
    m.gamg_setup(**ONE_SWEEP, **hier)
    g = O.Gamg(A, **hier)
    assert m.layout(0)["compressed"] is False and g.level(1).n > 300000
    assert m.downleg(0) == ("scaled_slices", 0)
    r = np.random.default_rng(45).standard_normal(c.n_cells)
    e = m.vcycle(_t(r), **ONE_SWEEP, **hier).cpu().numpy()
    ref = g.vcycle(r, n_pre=1, n_post=1, scale=False)
    assert np.linalg.norm(e - ref) <= 1e-11 * np.linalg.norm(ref)
    b = c.rhs[0]
    for tr in (False, True):
        if tr:
            x, st = m.adjoint(_t(b), solver="gamg", rel_tol=1e-8, history=100, **ONE_SWEEP,
                              **hier)
        else:
            x, st = m.gamg(_t(b), rel_tol=1e-8, history=100, **ONE_SWEEP, **hier)
        ref = g.solve(b, tol=1e-8, n_pre=1, n_post=1, scale=False, transpose=tr)
        assert st.converged and st.iterations == ref.iterations, tr
        assert hist_close(st.history, ref.history, 1e-8), tr
        assert np.linalg.norm(x.cpu().numpy() - ref.x) <= 1e-9 * np.linalg.norm(ref.x), tr
    m.close()


@pytest.mark.parametrize("name", ["ragged", "c5s", "nonsym", "c3s"])
def test_one_sweep_cycles_fuse_the_down_leg(name):
    """One Jacobi pre-sweep from zero and no correction scaling: each level's
    residual and restriction run as one product with R = P^T (I - w A D^-1).
    Against the oracle's two-step cycle: single V-cycles at two values of w
    (the second rebuilds R), CG + V-cycle forward, transposed and in mixed
    precision, standalone GAMG, and a V-cycle after new coefficients (R's
    values refreshed)."""
    from meshgen import assemble_diag
    c = _gamg_case(name)
    A = O.Ldu.from_case(c)
    m = _lib().from_case(c)
    g = O.Gamg(A)
    r = np.random.default_rng(41).standard_normal(c.n_cells)
    if c.singular:
        r -= r.mean()
    for omega in (0.75, 0.6, 0.75):
        e = m.vcycle(_t(r), omega=omega, **ONE_SWEEP).cpu().numpy()
        ref = g.vcycle(r, n_pre=1, n_post=1, omega=omega, scale=False)
        assert np.linalg.norm(e - ref) <= 1e-11 * np.linalg.norm(ref), omega
    b = c.rhs[0]
    m.gamg_setup(**ONE_SWEEP)  # a fresh hierarchy: R built again
    x, st = m.pcg(_t(b), precond=2, rel_tol=1e-8, history=500)
    ref = g.pcg(b, tol=1e-8, n_pre=1, n_post=1)
    assert st.converged and st.iterations == ref.iterations
    assert hist_close(st.history, ref.history, 1e-8)
    xg, xr = x.cpu().numpy(), ref.x
    if c.singular:
        xg, xr = xg - xg.mean(), xr - xr.mean()
    assert np.linalg.norm(xg - xr) <= 1e-9 * np.linalg.norm(xr)
    xt, stt = m.adjoint(_t(b), solver="pcg", precond=2, rel_tol=1e-8)
    reft = g.pcg(b, tol=1e-8, n_pre=1, n_post=1, transpose=True)
    assert stt.converged and stt.iterations == reft.iterations
    assert np.linalg.norm(b - O.tmul(A, xt.cpu().numpy())) <= 1e-8 * np.linalg.norm(b)
    # the transposed FP32 cycle (R's A^T values in FP32) inside FP64 refinement
    xtm, stm = m.adjoint(_t(b), solver="pcg", precond=2, rel_tol=1e-12, precision="mixed")
    assert stm.converged
    assert np.linalg.norm(b - O.tmul(A, xtm.cpu().numpy())) <= 1e-12 * np.linalg.norm(b)
    xm, sm = m.pcg(_t(b), precond=2, rel_tol=1e-12, precision="mixed")
    assert sm.converged and true_res(c, xm.cpu().numpy()) <= 1e-12
    if name in ("ragged", "nonsym"):  # standalone GAMG converges here without scaling
        xs, ss = m.gamg(_t(b), rel_tol=1e-8, history=300, **ONE_SWEEP)
        refs = g.solve(b, tol=1e-8, n_pre=1, n_post=1, scale=False)
        assert ss.converged and ss.iterations == refs.iterations
        assert hist_close(ss.history, refs.history)
    if name == "c5s":  # new coefficients on the same aggregation
        a2 = c.upper * np.exp(0.3 * np.random.default_rng(42).standard_normal(c.n_faces))
        d2 = assemble_diag(c.n_cells, c.owner, c.neighbour, a2, a2, c.meta["a_boundary"])
        m.set_coeffs(_t(d2), _t(a2), _t(a2))
        g.set_values(d2, a2, a2)
        e = m.vcycle(_t(r), **ONE_SWEEP).cpu().numpy()
        ref = g.vcycle(r, n_pre=1, n_post=1, scale=False)
        assert np.linalg.norm(e - ref) <= 1e-11 * np.linalg.norm(ref)
    m.close()


def test_one_sweep_cycle_on_a_level_above_the_fused_correction_size():
    """56^3 = 175,616 cells, above the size where the coarse level applies the
    correction itself: level 0's first sweep is then formed by the correction
    kernel.  CG + V-cycle against the oracle, forward and transposed."""
    c = box_case(56, 56, 56, coeff="lognormal", nonsym=0.2, dirichlet_x0=1.0, seed=43)
    A = O.Ldu.from_case(c)
    g = O.Gamg(A)
    m = _lib().from_case(c)
    m.gamg_setup(**ONE_SWEEP)
    b = c.rhs[0]
    x, st = m.pcg(_t(b), precond=2, rel_tol=1e-8, history=500)
    ref = g.pcg(b, tol=1e-8, n_pre=1, n_post=1)
    assert st.converged and st.iterations == ref.iterations
    assert hist_close(st.history, ref.history, 1e-8)
    assert np.linalg.norm(x.cpu().numpy() - ref.x) <= 1e-9 * np.linalg.norm(ref.x)
    xt, stt = m.adjoint(_t(b), solver="pcg", precond=2, rel_tol=1e-8)
    reft = g.pcg(b, tol=1e-8, n_pre=1, n_post=1, transpose=True)
    assert stt.converged and stt.iterations == reft.iterations
    assert np.linalg.norm(b - O.tmul(A, xt.cpu().numpy())) <= 1e-8 * np.linalg.norm(b)
    for tr, solve in ((False, m.pcg), (True, lambda v, **kw: m.adjoint(v, solver="pcg", **kw))):
        xm, sm = solve(_t(b), precond=2, rel_tol=1e-12, precision="mixed")
        xm = xm.cpu().numpy()
        res = b - (O.tmul(A, xm) if tr else O.amul(A, xm))
        assert sm.converged and np.linalg.norm(res) <= 1e-12 * np.linalg.norm(b), tr
    m.close()


def test_set_coeffs_recomputes_cached_hierarchy():
    from meshgen import assemble_diag
    c = _gamg_case("c5s")
    m = _lib().from_case(c)
    m.gamg_setup()
    a2 = c.upper * np.exp(0.3 * np.random.default_rng(5).standard_normal(c.n_faces))
    d2 = assemble_diag(c.n_cells, c.owner, c.neighbour, a2, a2, c.meta["a_boundary"])
    m.set_coeffs(_t(d2), _t(a2), _t(a2))
    g = O.Gamg(O.Ldu.from_case(c))
    g.set_values(d2, a2, a2)
    assert m.n_levels() == g.n_levels
    for l in range(g.n_levels):
        got = m.level(l)
        ref = g.level(l)
        for k, rv in (("diag", ref.diag), ("upper", ref.upper), ("lower", ref.lower)):
            assert np.array_equal(got[k].cpu().numpy(), rv), (l, k)
    A2 = O.Ldu(c.n_cells, c.owner, c.neighbour, d2, a2, a2)
    x = np.random.default_rng(6).standard_normal(c.n_cells)
    assert np.array_equal(m.amul(_t(x)).cpu().numpy(), O.amul(A2, x))
    xs, st = m.gamg(_t(c.rhs[0]))
    ref = g.solve(c.rhs[0])
    assert st.iterations == ref.iterations
    assert np.linalg.norm(xs.cpu().numpy() - ref.x) <= 1e-10 * np.linalg.norm(ref.x)


def test_autograd_matches_oracle_and_finite_differences():
    from meshgen import assemble_diag
    from paper_2512_22215_amd import ldu_solve
    c = box_case(9, 8, 7, coeff="lognormal", dirichlet_x0=2.0, seed=11)
    ab = np.where(np.arange(c.n_cells) % 9 == 0, 2.0, 0.0)
    xt = np.random.default_rng(12).standard_normal(c.n_cells)
    m = _lib().from_case(c)
    a = _t(c.upper).requires_grad_(True)
    b = _t(c.rhs[0]).requires_grad_(True)
    own = torch.from_numpy(c.owner.astype(np.int64)).cuda()
    nb = torch.from_numpy(c.neighbour.astype(np.int64)).cuda()

    def assemble(a):
        d = -(torch.zeros(c.n_cells, dtype=torch.float64, device="cuda")
              .index_add(0, own, a).index_add(0, nb, a)) - _t(ab)
        return d

    x = ldu_solve(assemble(a), a, a, b, m, "pcg", rel_tol=1e-13)
    loss = 0.5 * torch.sum((x - _t(xt)) ** 2)
    loss.backward()
    ga = a.grad.cpu().numpy()
    xn = x.detach().cpu().numpy()
    # oracle adjoint gradient for the symmetric face coefficient
    A = O.Ldu(c.n_cells, c.owner, c.neighbour, assemble_diag(c.n_cells, c.owner, c.neighbour,
                                                             c.upper, c.upper, ab),
              c.upper, c.upper)
    lam = O.pcg(A, xn - xt, tol=1e-13, transpose=True).x
    closed = (lam[c.owner] - lam[c.neighbour]) * (xn[c.owner] - xn[c.neighbour])
    assert np.allclose(ga, closed, rtol=1e-8, atol=1e-10 * np.abs(closed).max())
    assert np.linalg.norm(b.grad.cpu().numpy() - lam) <= 1e-9 * np.linalg.norm(lam)

    from tests.dense_ref import dense

    def L(av):
        # dense LU: loss evaluations accurate to ~1e-16 relative, so the
        # central difference resolves the gradient to ~1e-7
        d = assemble_diag(c.n_cells, c.owner, c.neighbour, av, av, ab)
        xx = np.linalg.solve(dense(c.n_cells, c.owner, c.neighbour, d, av, av), c.rhs[0])
        return 0.5 * np.sum((xx - xt) ** 2)

    # relative step 1e-4: truncation O(h^2) and roundoff (eps L / h) both stay
    # below 1e-7 of the gradient here; at 1e-6 the roundoff of L alone
    # reaches 5e-5 on faces with small gradients
    for f in np.random.default_rng(13).choice(c.n_faces, 5, replace=False):
        h = 1e-4 * c.upper[f]
        ap = c.upper.copy(); ap[f] += h
        am = c.upper.copy(); am[f] -= h
        fd = (L(ap) - L(am)) / (2 * h)
        assert abs(fd - ga[f]) <= 1e-5 * max(abs(ga[f]), 1e-3 * np.abs(ga).max())


def test_oversized_coarsest_level_is_refused_at_setup():
    """A hierarchy cut off above 8192 coarsest cells (here by max_levels) is
    refused before any solve; the handle stays usable."""
    from paper_2512_22215_amd import LduError
    from paper_2512_22215_amd.ldu import LDU_ERR_LIMIT
    c = _gamg_case("c5s")
    m = _lib().from_case(c)
    with pytest.raises(LduError) as e:
        m.gamg_setup(max_levels=2)
    assert e.value.code == LDU_ERR_LIMIT
    x, st = m.gamg(_t(c.rhs[0]), rel_tol=1e-8)
    assert st.converged and true_res(c, x.cpu().numpy()) <= 1e-8


@pytest.mark.parametrize("name", ["nonsym", "c5u"])
@pytest.mark.parametrize("precond", [0, 1])
def test_pbicg_matches_oracle(name, precond):
    """PBiCG (fused Amul + Tmul) against the oracle: forward and transposed
    solves.  The products are bit-exact and only the dot products' summation
    orders differ, so the first ten residuals agree to 1e-11 (measured: 2e-13
    at most); later, BiCG's near-breakdowns (it minimises nothing) amplify
    those roundings, and a residual that crosses the tolerance within that
    rounding may stop one iteration earlier or later (measured: 0 or 1 on
    every case), so the paths are compared by iteration count (within one)
    and by the solutions (both at the tolerance, and within 1e-8 of each
    other)."""
    from meshgen import config_case
    c = CASES["nonsym"] if name == "nonsym" else config_case("c5u", n=24)
    A = O.Ldu.from_case(c)
    m = _lib().from_case(c)
    for tr in (False, True):
        if tr:
            lam, st = m.adjoint(_t(c.rhs[0]), solver="pbicg", rel_tol=1e-10, precond=precond,
                                history=2000)
            xg = lam.cpu().numpy()
        else:
            x, st = m.pbicg(_t(c.rhs[0]), rel_tol=1e-10, precond=precond, history=2000)
            xg = x.cpu().numpy()
        ref = O.pbicg(A, c.rhs[0], tol=1e-10, precond=bool(precond), transpose=tr)
        assert ref.status == O.OK and st.converged
        assert abs(st.iterations - ref.iterations) <= 1, (st.iterations, ref.iterations)
        h = np.asarray(st.history)
        dev = np.abs(h[:11] - ref.history[:11]) / ref.history[:11]
        print(f"{name} precond {precond} transpose {tr}: {st.iterations} vs "
              f"{ref.iterations} iterations, history deviation over 10 steps {dev.max():.2e}")
        assert dev.max() <= 1e-11
        bt = O.tmul(A, xg) if tr else O.amul(A, xg)
        assert np.linalg.norm(c.rhs[0] - bt) <= 1e-10 * np.linalg.norm(c.rhs[0])
        assert np.linalg.norm(xg - ref.x) <= 1e-8 * np.linalg.norm(ref.x)


def test_pbicg_equals_pcg_on_symmetric_and_rejects_bad_options():
    from paper_2512_22215_amd import LduError
    c = CASES["c1"]
    m = _lib().from_case(c)
    xb, sb = m.pbicg(_t(c.rhs[0]), rel_tol=1e-8)
    xc, sc = m.pcg(_t(c.rhs[0]), rel_tol=1e-8)
    assert sb.iterations == sc.iterations
    assert np.linalg.norm((xb - xc).cpu().numpy()) <= 1e-12 * np.linalg.norm(xc.cpu().numpy())
    for bad in (dict(precond=2), dict(precision="mixed")):
        with pytest.raises(LduError):
            m.pbicg(_t(c.rhs[0]), **bad)


def test_autograd_pbicg_nonsymmetric_matches_dense():
    """Gradients through a non-symmetric solve (PBiCG forward and adjoint)
    against dense linear algebra."""
    from meshgen import config_case
    from paper_2512_22215_amd import ldu_solve
    c = config_case("c5u", n=9)
    m = _lib().from_case(c)
    d = _t(c.diag).requires_grad_(True)
    u = _t(c.upper).requires_grad_(True)
    lo = _t(c.lower).requires_grad_(True)
    b = _t(c.rhs[0]).requires_grad_(True)
    xt = np.random.default_rng(13).standard_normal(c.n_cells)
    x = ldu_solve(d, u, lo, b, m, "pbicg", rel_tol=1e-13)
    loss = 0.5 * torch.sum((x - _t(xt)) ** 2)
    loss.backward()
    D = np.zeros((c.n_cells, c.n_cells))
    D[np.arange(c.n_cells), np.arange(c.n_cells)] = c.diag
    D[c.owner, c.neighbour] = c.upper
    D[c.neighbour, c.owner] = c.lower
    xd = np.linalg.solve(D, c.rhs[0])
    lam = np.linalg.solve(D.T, xd - xt)
    assert np.linalg.norm(x.detach().cpu().numpy() - xd) <= 1e-10 * np.linalg.norm(xd)
    for got, want in ((b.grad, lam), (d.grad, -lam * xd),
                      (u.grad, -lam[c.owner] * xd[c.neighbour]),
                      (lo.grad, -lam[c.neighbour] * xd[c.owner])):
        g = got.cpu().numpy()
        assert np.linalg.norm(g - want) <= 1e-9 * np.linalg.norm(want)


def _assembly_matrix(g):
    """A handle on the assembly mesh, created with placeholder coefficients."""
    from paper_2512_22215_amd import LduMatrix
    nf = g["owner"].size
    return LduMatrix(g["n"], _t(g["owner"].astype(np.int32)), _t(g["neighbour"].astype(np.int32)),
                     _t(-6.0 * np.ones(g["n"])), _t(np.ones(nf)), _t(np.ones(nf)), device="cuda")


def test_pressure_assembly_bit_exact_and_feeds_the_solvers():
    from meshgen import c3_assembly_inputs
    g = c3_assembly_inputs(n=24, nxy=10)
    m = _assembly_matrix(g)
    m.gamg_setup()  # a cached hierarchy must pick up the new values
    args = [g[k] for k in ("gamma", "weights", "mag_sf", "delta")]
    b, (d, u, lo) = m.assemble_pressure(*args, diag_bc=g["diag_bc"], phi=g["phi"],
                                        b_bc=g["b_bc"], out_coeffs=True)
    rd, ru, rl, rb = O.assemble_pressure(g["n"], g["owner"], g["neighbour"], *args,
                                         g["diag_bc"], g["phi"], g["b_bc"])
    for got, want in ((d, rd), (u, ru), (lo, rl), (b, rb)):
        assert np.array_equal(got.cpu().numpy(), want)
    A = O.Ldu(g["n"], g["owner"], g["neighbour"], rd, ru, rl)
    # the handle now holds the assembled matrix: products, hierarchy, solve
    x = np.random.default_rng(21).standard_normal(g["n"])
    assert np.array_equal(m.amul(_t(x)).cpu().numpy(), O.amul(A, x))
    # the cached aggregation is the placeholder matrix's; its Galerkin values
    # are recomputed from the assembled ones
    nf = g["owner"].size
    ref = O.Gamg(O.Ldu(g["n"], g["owner"], g["neighbour"], -6.0 * np.ones(g["n"]),
                       np.ones(nf), np.ones(nf)))
    ref.set_values(rd, ru, rl)
    assert m.n_levels() == ref.n_levels
    for l in range(ref.n_levels):
        lv = m.level(l)
        assert np.array_equal(lv["diag"].cpu().numpy(), ref.level(l).diag), l
        assert np.array_equal(lv["upper"].cpu().numpy(), ref.level(l).upper), l
    rhs = rb + 0.1 * np.random.default_rng(22).standard_normal(g["n"])
    xs, st = m.pcg(_t(rhs), precond=2, rel_tol=1e-8, max_iter=2000)
    assert st.converged
    assert np.linalg.norm(rhs - O.amul(A, xs.cpu().numpy())) <= 1e-8 * np.linalg.norm(rhs)
    # optional inputs: no boundary terms, no right-hand side
    assert m.assemble_pressure(*args) is None
    rd0, _, _, _ = O.assemble_pressure(g["n"], g["owner"], g["neighbour"], *args)
    _, (d0, _, _) = m.assemble_pressure(*args, out_coeffs=True)
    assert np.array_equal(d0.cpu().numpy(), rd0)
    with pytest.raises(ValueError):
        m.assemble_pressure(g["gamma"][:-1], *args[1:])


@pytest.mark.parametrize("n", [1, 70])
def test_solvers_on_matrices_without_faces(n):
    """Degenerate inputs: one cell, or a diagonal matrix with no faces (one
    GAMG level, which is its own coarsest level; for 70 cells the workgroup
    coarsest kernel).  Every solver returns D^-1 b; the assembly leaves
    diag = -diag_bc and b = b_bc."""
    from meshgen.boxes import LduCase
    e = np.zeros(0, np.int32)
    d = -1.0 - np.arange(n, dtype=np.float64)
    b = np.random.default_rng(31).standard_normal(n)
    c = LduCase("diag", n, e, e.copy(), d, np.zeros(0), np.zeros(0), [b], False)
    m = _lib().from_case(c)
    want = b / d
    for x, st in (m.pcg(_t(b)), m.pcg(_t(b), precond=2), m.gamg(_t(b)), m.pbicg(_t(b)),
                  m.pcg(_t(b), precision="mixed"), m.gamg(_t(b), precision="mixed")):
        assert st.converged
        assert np.allclose(x.cpu().numpy(), want, rtol=1e-8, atol=0)
    assert m.n_levels() == 1
    bc = np.abs(b)
    bb, (dd, uu, ll) = m.assemble_pressure(np.ones(n), np.zeros(0), np.zeros(0), np.zeros(0),
                                           diag_bc=bc, phi=np.zeros(0), b_bc=b,
                                           out_coeffs=True)
    assert np.array_equal(dd.cpu().numpy(), -bc) and np.array_equal(bb.cpu().numpy(), b)
    assert uu.numel() == 0 and ll.numel() == 0


def test_create_rejects_duplicate_and_out_of_range_faces():
    """Addressing errors the validator must catch before any kernel indexes
    with the faces (it reads only owner[f], neighbour[f] and face f - 1)."""
    from paper_2512_22215_amd import LduError
    c = CASES["ragged"]
    LduMatrix = _lib()
    f = 40
    own = np.insert(c.owner, f, c.owner[f])          # a duplicate of face f
    nb = np.insert(c.neighbour, f, c.neighbour[f])
    up = np.insert(c.upper, f, 1.0)
    lo = np.insert(c.lower, f, 1.0)
    bad = [(own, nb, up, lo)]
    nb2 = c.neighbour.copy(); nb2[-1] = c.n_cells      # neighbour out of range
    bad.append((c.owner, nb2, c.upper, c.lower))
    own3 = c.owner.copy(); own3[0] = -1                 # negative owner
    bad.append((own3, c.neighbour, c.upper, c.lower))
    nb4 = c.neighbour.copy(); nb4[7] = 2 ** 31 - 1      # far out of range
    bad.append((c.owner, nb4, c.upper, c.lower))
    for k, (o, n, u, l) in enumerate(bad):
        with pytest.raises(LduError) as e:
            LduMatrix(c.n_cells, o, n, c.diag, u, l)
        assert e.value.code == -2, k
    # the oracle's validator agrees
    for o, n, u, l in bad:
        assert O.validate(c.n_cells, o, n, c.diag, u, l) == O.ERR_ADDR


def test_nan_rhs_is_reported_by_every_solver():
    from paper_2512_22215_amd import LduError
    c = CASES["ragged"]
    m = _lib().from_case(c)
    m.gamg_setup(n_pre=1, n_post=1)
    b = c.rhs[0].copy()
    b[123] = np.nan
    runs = [(m.pcg, {}), (m.pcg, dict(precision="mixed")), (m.pcg, dict(precond=2)),
            (m.pcg, dict(precond=2, precision="mixed")), (m.gamg, dict(n_pre=1, n_post=1)),
            (m.gamg, dict(n_pre=1, n_post=1, precision="mixed")), (m.pbicg, {})]
    for fn, kw in runs:
        with pytest.raises(LduError) as e:
            fn(_t(b), **kw)
        assert e.value.code == -3, (fn.__name__, kw)
    # a NaN in the initial guess as well
    x0 = np.zeros(c.n_cells); x0[5] = np.inf
    with pytest.raises(LduError) as e:
        m.pcg(_t(c.rhs[0]), x0=_t(x0))
    assert e.value.code == -3
    # the handle is not poisoned by these errors
    x, st = m.pcg(_t(c.rhs[0]), rel_tol=1e-8)
    assert st.converged
    m.close()


def test_inconsistent_singular_rhs_is_not_converged():
    """A pure zero-gradient (singular) system with a right-hand side of
    nonzero mean has no solution: every solver runs out of its budget and
    returns LDU_NOT_CONVERGED with the last iterate, as the oracle does; the
    true residual stays above the least-squares bound |mean(b)| sqrt(n)/||b||."""
    c = box_case(9, 8, 7, coeff="lognormal", seed=3)
    b = c.rhs[0] + 0.3
    A = O.Ldu.from_case(c)
    bound = abs(b.mean()) * np.sqrt(c.n_cells) / np.linalg.norm(b)
    m = _lib().from_case(c)
    m.gamg_setup(n_coarsest=10, n_pre=1, n_post=1)
    g = O.Gamg(A, n_coarsest=10)
    runs = [("pcg", m.pcg(_t(b), max_iter=50), O.pcg(A, b, max_iter=50)),
            ("gamg", m.gamg(_t(b), max_cycles=30, n_coarsest=10, n_pre=1, n_post=1),
             g.solve(b, max_cycles=30, n_pre=1, n_post=1)),
            ("mixed", m.pcg(_t(b), precision="mixed", max_refine=3),
             O.pcg_mixed(A, b, max_refine=3))]
    for name, (x, st), ref in runs:
        print(f"{name}: status {st.status} it {st.iterations} ref {ref.status} "
              f"it {ref.iterations} residual {st.final_residual:.3e}", flush=True)
        assert st.status == 1 and ref.status == O.NOT_CONVERGED and not st.converged, name
        assert np.all(np.isfinite(x.cpu().numpy()))
        assert st.final_residual >= bound * (1 - 1e-9)
    assert runs[0][1][1].iterations == 50 == runs[0][2].iterations
    assert runs[1][1][1].iterations == 30 == runs[1][2].iterations
    m.close()


@pytest.mark.parametrize("rounds", [1, 2, 16])
def test_match_round_cap_matches_oracle(rounds):
    """On a chain where every handshake round pairs one pair per block, the
    cap on matching rounds binds; aggregates equal the oracle's."""
    from tests.test_oracle_pins import _sawtooth_chain
    n, own, nb, d, a = _sawtooth_chain()
    m = _lib()(n, own, nb, d, a, a)
    m.gamg_setup(n_coarsest=2, max_levels=2, match_rounds=rounds)
    g = O.Gamg(O.Ldu(n, own, nb, d, a, a), n_coarsest=2, max_levels=2, match_rounds=rounds)
    assert np.array_equal(m.level(0)["agg"].cpu().numpy(), g.level(0).agg)
    m.close()


def test_autograd_two_forwards_share_a_matrix():
    """Two solves on one LduMatrix with different coefficients, then one
    backward through both: each backward solves with its own coefficients."""
    from meshgen import assemble_diag
    from paper_2512_22215_amd import ldu_solve
    c = box_case(8, 7, 6, coeff="lognormal", dirichlet_x0=2.0, seed=21)
    ab = np.where(np.arange(c.n_cells) % 8 == 0, 2.0, 0.0)
    m = _lib().from_case(c)
    own = torch.from_numpy(c.owner.astype(np.int64)).cuda()
    nb = torch.from_numpy(c.neighbour.astype(np.int64)).cuda()

    def assemble(a):
        return -(torch.zeros(c.n_cells, dtype=torch.float64, device="cuda")
                 .index_add(0, own, a).index_add(0, nb, a)) - _t(ab)

    a1 = _t(c.upper).requires_grad_(True)
    a2 = _t(c.upper * 1.7 + 0.1).requires_grad_(True)
    b = _t(c.rhs[0])
    x1 = ldu_solve(assemble(a1), a1, a1, b, m, "pcg", rel_tol=1e-13)
    x2 = ldu_solve(assemble(a2), a2, a2, b, m, "pcg", rel_tol=1e-13)
    (0.5 * torch.sum(x1 ** 2) + torch.sum(x2)).backward()
    for a, x, g in ((a1, x1, x1.detach()), (a2, x2, torch.ones_like(x2))):
        av = a.detach().cpu().numpy()
        A = O.Ldu(c.n_cells, c.owner, c.neighbour,
                  assemble_diag(c.n_cells, c.owner, c.neighbour, av, av, ab), av, av)
        xn = x.detach().cpu().numpy()
        lam = O.pcg(A, g.cpu().numpy(), tol=1e-13, transpose=True).x
        closed = (lam[c.owner] - lam[c.neighbour]) * (xn[c.owner] - xn[c.neighbour])
        assert np.allclose(a.grad.cpu().numpy(), closed, rtol=1e-8,
                           atol=1e-10 * np.abs(closed).max())
    m.close()


def test_autograd_raises_when_a_solve_does_not_converge():
    from paper_2512_22215_amd import LduError, ldu_solve
    c = CASES["ragged"]
    m = _lib().from_case(c)
    a = _t(c.upper).requires_grad_(True)
    with pytest.raises(LduError) as e:
        ldu_solve(_t(c.diag), a, a, _t(c.rhs[0]), m, "pcg", rel_tol=1e-12, max_iter=3)
    assert e.value.code == 1
    m.close()
