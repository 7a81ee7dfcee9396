"""Seeded random configurations of the GAMG path against the CPU oracle.

Each configuration draws a box mesh (3 to 40 cells per side, at most about
30,000 cells), a coefficient model (uniform or log-normal; symmetric or
not), an optional random renumbering, and a cycle (pairwise or aggressive
agglomeration from level 0, 1 or 2; damped Jacobi or two-stage Gauss-Seidel;
diagonal or DIC coarsest; 1 or 2 sweeps; correction scaling on or off).  The
draws come from numpy's default_rng with the configuration's index as seed,
so every run checks the same configurations.  Bars, as in the fixed parity
tests: aggregates integer-equal on every level, one V-cycle within 1e-11,
standalone GAMG (forward, and transposed on non-symmetric matrices) and, on
symmetric matrices, CG + V-cycle with equal iteration counts and solutions
within 1e-9, and the mixed CG + V-cycle refined to 1e-10.
"""
import numpy as np
import pytest

import oracle as O
from meshgen import box_case, random_order, relabel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N_CONFIGS = 48


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def draw(seed):
    """The configuration of one seed: the case and the cycle options."""
    rng = np.random.default_rng(seed)
    while True:
        nx, ny, nz = (int(v) for v in rng.integers(3, 41, 3))
        if nx * ny * nz <= 30000:
            break
    nonsym = float(rng.choice([0.0, 0.0, 0.5]))
    coeff = str(rng.choice(["uniform", "lognormal"]))
    c = box_case(nx, ny, nz, coeff=coeff, nonsym=nonsym, dirichlet_x0=1.0,
                 seed=int(rng.integers(1 << 30)))
    if rng.random() < 0.5:
        c = relabel(c, random_order(c.n_cells, rng))
    hier = {}
    passes = int(rng.choice([1, 2, 3]))
    if passes > 1:
        hier = dict(passes=passes, aggressive_from=int(rng.integers(0, 3)))
    cycle = dict(smoother=str(rng.choice(["jacobi", "jacobi", "gs2"])),
                 coarsest=str(rng.choice(["diag", "dic"])))
    if cycle["smoother"] == "gs2":
        cycle["gs_inner"] = int(rng.integers(1, 3))
    sweeps = int(rng.choice([1, 2]))
    scale = int(rng.integers(0, 2))
    return c, nonsym > 0, hier, cycle, sweeps, scale


def describe(seed):
    c, nonsym, hier, cycle, sweeps, scale = draw(seed)
    return (f"seed {seed}: {c.n_cells} cells, nonsym {nonsym}, {hier or 'pairwise'}, "
            f"{cycle}, sweeps {sweeps}, scale {scale}")


@pytest.mark.parametrize("seed", range(N_CONFIGS))
def test_random_configuration(seed):
    from paper_2512_22215_amd import LduMatrix
    print(describe(seed), flush=True)
    c, nonsym, hier, cycle, sweeps, scale = draw(seed)
    A = O.Ldu.from_case(c)
    g = O.Gamg(A, **hier, **cycle)
    m = LduMatrix.from_case(c)
    opts = dict(n_pre=sweeps, n_post=sweeps, scale_correction=scale, **hier, **cycle)
    m.gamg_setup(**opts)
    assert m.n_levels() == g.n_levels
    for lev in range(g.n_levels - 1):
        assert np.array_equal(m.level(lev)["agg"].cpu().numpy(), g.level(lev).agg), lev
    r = np.random.default_rng(1000 + seed).standard_normal(c.n_cells)
    e = m.vcycle(_t(r), **opts).cpu().numpy()
    ref = g.vcycle(r, n_pre=sweeps, n_post=sweeps, scale=bool(scale))
    assert np.linalg.norm(e - ref) <= 1e-11 * np.linalg.norm(ref)
    b = c.rhs[0]
    for tr in ((False, True) if nonsym else (False,)):
        rs = g.solve(b, tol=1e-8, max_cycles=100, n_pre=sweeps, n_post=sweeps,
                     scale=bool(scale), transpose=tr)
        if tr:
            x, st = m.adjoint(_t(b), solver="gamg", rel_tol=1e-8, max_cycles=100, **opts)
        else:
            x, st = m.gamg(_t(b), rel_tol=1e-8, max_cycles=100, **opts)
        assert st.iterations == rs.iterations, (tr, st.iterations, rs.iterations)
        assert st.converged == (rs.status == O.OK), tr
        if st.converged:
            assert np.linalg.norm(x.cpu().numpy() - rs.x) <= 1e-9 * np.linalg.norm(rs.x), tr
    if not nonsym:
        copts = dict(opts, scale_correction=0)
        m.gamg_setup(**copts)
        x, st = m.pcg(_t(b), precond=2, rel_tol=1e-8)
        rp = g.pcg(b, tol=1e-8, n_pre=sweeps, n_post=sweeps)
        assert st.converged and rp.status == O.OK
        assert st.iterations == rp.iterations, (st.iterations, rp.iterations)
        assert np.linalg.norm(x.cpu().numpy() - rp.x) <= 1e-9 * np.linalg.norm(rp.x)
        xm, sm = m.pcg(_t(b), precond=2, rel_tol=1e-10, precision="mixed")
        assert sm.converged
        res = np.linalg.norm(b - O.amul(A, xm.cpu().numpy())) / np.linalg.norm(b)
        assert res <= 1e-10, res
    m.close()


def draw_mesh(seed):
    """A random mesh of the product tests: box sizes 1 to 60 per side (at
    most 60,000 cells), symmetric or not, renumbered or not."""
    rng = np.random.default_rng(5000 + seed)
    while True:
        nx, ny, nz = (int(v) for v in rng.integers(1, 61, 3))
        if nx * ny * nz <= 60000:
            break
    nonsym = float(rng.choice([0.0, 0.5]))
    c = box_case(nx, ny, nz, coeff=str(rng.choice(["uniform", "lognormal"])), nonsym=nonsym,
                 dirichlet_x0=1.0, seed=int(rng.integers(1 << 30)))
    if rng.random() < 0.5:
        c = relabel(c, random_order(c.n_cells, rng))
    return c, nonsym > 0, rng


@pytest.mark.parametrize("seed", range(N_CONFIGS))
def test_random_products_and_krylov(seed):
    """Amul, Tmul and the FP32 Amul bit-exact, the coefficient gradients
    bit-exact given lambda and x, diagonal PCG (symmetric meshes: equal
    counts, solutions within 1e-10) and PBiCG (non-symmetric meshes: counts
    within one, solutions within 1e-8) on random meshes."""
    from paper_2512_22215_amd import LduMatrix
    c, nonsym, rng = draw_mesh(seed)
    print(f"seed {seed}: {c.n_cells} cells, {c.n_faces} faces, nonsym {nonsym}", flush=True)
    A = O.Ldu.from_case(c)
    m = LduMatrix.from_case(c)
    x = rng.standard_normal(c.n_cells)
    assert np.array_equal(m.amul(_t(x)).cpu().numpy(), O.amul(A, x))
    assert np.array_equal(m.tmul(_t(x)).cpu().numpy(), O.tmul(A, x))
    x32 = x.astype(np.float32)
    assert np.array_equal(m.amul_f32(_t(x32)).cpu().numpy(), O.amul_f32(A, x32))
    lam = rng.standard_normal(c.n_cells)
    gd, gu, gl = (t.cpu().numpy() for t in m.coeff_grad(_t(lam), _t(x)))
    rd, ru, rl = O.coeff_grad(A, lam, x)
    assert np.array_equal(gd, rd) and np.array_equal(gu, ru) and np.array_equal(gl, rl)
    b = c.rhs[0]
    if not nonsym:
        xg, st = m.pcg(_t(b), precond=1, rel_tol=1e-10)
        ref = O.pcg(A, b, tol=1e-10)
        assert st.converged and ref.status == O.OK
        assert st.iterations == ref.iterations, (st.iterations, ref.iterations)
        assert np.linalg.norm(xg.cpu().numpy() - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
    else:
        xg, st = m.pbicg(_t(b), precond=1, rel_tol=1e-10)
        ref = O.pbicg(A, b, tol=1e-10)
        assert st.converged and ref.status == O.OK
        assert abs(st.iterations - ref.iterations) <= 1, (st.iterations, ref.iterations)
        assert np.linalg.norm(xg.cpu().numpy() - ref.x) <= 1e-8 * np.linalg.norm(ref.x)
    m.close()


@pytest.mark.parametrize("seed", range(16))
def test_random_differentiable_solve(seed):
    """The differentiable solve on random small meshes (at most 400 cells,
    symmetric or not, renumbered or not): x and the gradients of
    L = 0.5 |x - x_t|^2 with respect to diag, upper, lower and b through the
    autograd Function, against dense float64 algebra on the CPU
    (x = A^-1 b; lambda = A^-T (x - x_t); dL/db = lambda; dL/dA = -lambda x^T
    read at the diagonal and at each face's two entries), for the CG + V-cycle
    in FP64 and in the mixed form (symmetric meshes) and PBiCG in FP64
    (non-symmetric meshes; PBiCG has no mixed form)."""
    from paper_2512_22215_amd import LduMatrix, ldu_solve
    rng = np.random.default_rng(9000 + seed)
    while True:
        nx, ny, nz = (int(v) for v in rng.integers(1, 12, 3))
        if 2 <= nx * ny * nz <= 400:
            break
    nonsym = bool(rng.random() < 0.5)
    c = box_case(nx, ny, nz, coeff="lognormal", nonsym=0.5 if nonsym else 0.0,
                 dirichlet_x0=1.0, seed=int(rng.integers(1 << 30)))
    if rng.random() < 0.5:
        c = relabel(c, random_order(c.n_cells, rng))
    n, own, nb = c.n_cells, c.owner, c.neighbour
    A = np.diag(c.diag.astype(np.float64))
    A[own, nb] = c.upper
    A[nb, own] = c.lower
    b = c.rhs[0]
    xt = rng.standard_normal(n)
    x_ref = np.linalg.solve(A, b)
    lam = np.linalg.solve(A.T, x_ref - xt)
    gA = -np.outer(lam, x_ref)
    ref = {"diag": np.diag(gA), "upper": gA[own, nb], "lower": gA[nb, own], "b": lam}
    m = LduMatrix.from_case(c)
    method = "pbicg" if nonsym else "pcg"
    for prec in (("fp64",) if nonsym else ("fp64", "mixed")):
        opts = dict(rel_tol=1e-13, precision=prec)
        if method == "pcg":
            opts["precond"] = 2
        leaves = {k: _t(v).requires_grad_() for k, v in
                  (("diag", c.diag), ("upper", c.upper), ("lower", c.lower), ("b", b))}
        x = ldu_solve(leaves["diag"], leaves["upper"], leaves["lower"], leaves["b"], m,
                      method, **opts)
        loss = 0.5 * ((x - _t(xt)) ** 2).sum()
        loss.backward()
        xg = x.detach().cpu().numpy()
        assert np.linalg.norm(xg - x_ref) <= 1e-10 * np.linalg.norm(x_ref), prec
        for k, v in ref.items():
            got = leaves[k].grad.cpu().numpy()
            assert np.linalg.norm(got - v) <= 1e-9 * np.linalg.norm(v), (prec, k)
    m.close()


@pytest.mark.parametrize("seed", range(16))
def test_random_pressure_assembly(seed):
    """Pressure assembly on random box meshes (1 to 40 cells per side,
    renumbered or not) with random inputs (gamma log-normal, weights in
    (0, 1), positive |S| and delta, random boundary coefficients, fluxes and
    sources): diag, upper, lower and b bit-exact against the oracle, then
    the handle's Amul bit-exact on the assembled matrix."""
    from paper_2512_22215_amd import LduMatrix
    rng = np.random.default_rng(7000 + seed)
    while True:
        nx, ny, nz = (int(v) for v in rng.integers(1, 41, 3))
        if 2 <= nx * ny * nz <= 40000:
            break
    c = box_case(nx, ny, nz, coeff="uniform", dirichlet_x0=1.0, seed=seed)
    if rng.random() < 0.5:
        c = relabel(c, random_order(c.n_cells, rng))
    n, nf = c.n_cells, c.n_faces
    gamma = np.exp(0.5 * rng.standard_normal(n))
    weights = rng.uniform(0.05, 0.95, nf)
    mag_sf = rng.uniform(0.5, 2.0, nf)
    delta = rng.uniform(0.5, 2.0, nf)
    diag_bc = np.where(rng.random(n) < 0.1, rng.uniform(0.5, 2.0, n), 0.0)
    phi = rng.standard_normal(nf)
    b_bc = np.where(rng.random(n) < 0.1, rng.standard_normal(n), 0.0)
    m = LduMatrix(n, _t(c.owner.astype(np.int32)), _t(c.neighbour.astype(np.int32)),
                  _t(-6.0 * np.ones(n)), _t(np.ones(nf)), _t(np.ones(nf)))
    b, (d, u, lo) = m.assemble_pressure(_t(gamma), _t(weights), _t(mag_sf), _t(delta),
                                        diag_bc=_t(diag_bc), phi=_t(phi), b_bc=_t(b_bc),
                                        out_coeffs=True)
    rd, ru, rl, rb = O.assemble_pressure(n, c.owner, c.neighbour, gamma, weights, mag_sf,
                                         delta, diag_bc, phi, b_bc)
    for got, want in ((d, rd), (u, ru), (lo, rl), (b, rb)):
        assert np.array_equal(got.cpu().numpy(), want)
    A = O.Ldu(n, c.owner, c.neighbour, rd, ru, rl)
    x = rng.standard_normal(n)
    assert np.array_equal(m.amul(_t(x)).cpu().numpy(), O.amul(A, x))
    m.close()
