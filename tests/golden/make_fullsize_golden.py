"""Write the full-size reference results, tests/golden/fullsize_<workload>.json,
from the CPU oracle only (test infrastructure: nothing here touches a GPU).

The GPU tests at full size compare their solves with these.  Storing whole
solution vectors (8M-17M doubles each) is not practical, so each result
keeps its iteration count, residual history, the 2-norm of x and x at
SAMPLES cell indices drawn by numpy's default_rng(SAMPLE_SEED) without
replacement (stored too).  The solver settings are the GPU tests':

  c3  200^3 graded hex (8M cells): CG preconditioned by one V-cycle
      (pairwise agglomeration, 1 + 1 Jacobi sweeps, omega 0.75, correction
      scaling off, diagonal-CG coarsest), FP64, x0 = 0, to 1e-8; and the same
      with three matching passes per level below level 1 (AGGRESSIVE).
  c4  256^3 RCM box (16.7M cells), three right-hand sides back to back, each
      warm-started from the previous solution: the same CG + V-cycle, and
      diagonal PCG, both FP64 to 1e-8.
  c5  100^3 box (1M cells): x = A^-1 b and lambda = A^-T (x - x_t) with the
      CG + V-cycle, x to 1e-13 and lambda to 1e-11 (the FP64 floor of the
      adjoint: ||A|| ||lambda|| is about 5e4 ||x - x_t||, so a recomputed
      residual carries rounding noise near 5e-12), the adjoint gradients of the symmetric face
      coefficients c_f (upper = lower = c_f, each end's diagonal -= c_f):
      dL/dc_f = (lambda_own - lambda_nb)(x_own - x_nb) at sampled faces and at
      the 20 seeded faces, and at those 20 faces central finite differences
      with a relative step of about 1e-6 (a power of two; exact perturbation
      and increment form, see the comment in run_c5).

Run: python tests/golden/make_fullsize_golden.py c3 c4 c5   (minutes each)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from meshgen import assemble_diag, config_case  # noqa: E402

SAMPLES = 4096
SAMPLE_SEED = 8701
AGGRESSIVE = {"passes": 3, "aggressive_from": 1}


def sample_indices(n, seed=SAMPLE_SEED, k=SAMPLES):
    return np.sort(np.random.default_rng(seed).choice(n, k, replace=False))


def vec_record(x, idx):
    return {"norm2": float(np.linalg.norm(x)), "sample": [float(v) for v in x[idx]]}


def solve_record(r, idx, seconds):
    return {"status": int(r.status), "iterations": int(r.iterations),
            "history": [float(v) for v in r.history],
            "true_residual": float(r.true_residual), "seconds": seconds,
            "x": vec_record(r.x, idx)}


def timed(fn):
    t0 = time.perf_counter()
    out = fn()
    return out, time.perf_counter() - t0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_c3():
    c = config_case("c3")
    A = O.Ldu.from_case(c)
    idx = sample_indices(c.n_cells)
    out = {"workload": "c3: 200^3 graded hex, 8,000,000 cells",
           "sample_seed": SAMPLE_SEED, "indices": idx.tolist()}
    # the pairwise hierarchy, and pairwise level 0 -> 1 followed by three
    # matching passes per level (aggregates of about eight cells below)
    for suffix, kw in (("", {}), ("_aggressive", AGGRESSIVE)):
        g, tb = timed(lambda: O.Gamg(A, **kw))
        log(f"c3{suffix}: GAMG build {tb:.1f} s, {g.n_levels} levels")
        r, ts = timed(lambda: g.pcg(c.rhs[0], tol=1e-8, n_pre=1, n_post=1))
        log(f"c3{suffix}: CG + V-cycle {r.iterations} iterations, {ts:.1f} s")
        out["levels" + suffix] = [g.level(k).n for k in range(g.n_levels)]
        out["pcg_gamg_fp64" + suffix] = solve_record(r, idx, ts)
        del g
    out["aggressive_settings"] = AGGRESSIVE
    return out


def run_c4():
    c = config_case("c4")
    A = O.Ldu.from_case(c)
    idx = sample_indices(c.n_cells)
    out = {"workload": "c4: 256^3 RCM box, 16,777,216 cells, three warm-started rhs",
           "sample_seed": SAMPLE_SEED, "indices": idx.tolist()}
    g, tb = timed(lambda: O.Gamg(A))
    log(f"c4: GAMG build {tb:.1f} s, {g.n_levels} levels")
    out["levels"] = [g.level(k).n for k in range(g.n_levels)]
    for label, solve in (("pcg_gamg_fp64", lambda b, x0: g.pcg(b, x0=x0, tol=1e-8, n_pre=1,
                                                                n_post=1)),
                         ("pcg_diag_fp64", lambda b, x0: O.pcg(A, b, x0=x0, tol=1e-8))):
        x = np.zeros(c.n_cells)
        runs = []
        for k, b in enumerate(c.rhs):
            r, ts = timed(lambda: solve(b, x))
            log(f"c4 {label} rhs {k}: {r.iterations} iterations, {ts:.1f} s")
            runs.append(solve_record(r, idx, ts))
            x = r.x
        out[label] = runs
    return out


def run_c5():
    c = config_case("c5")
    A = O.Ldu.from_case(c)
    ab = c.meta["a_boundary"]
    xt = c.meta["x_target"]
    b = c.rhs[0]
    idx = sample_indices(c.n_cells)
    fidx = sample_indices(c.n_faces, SAMPLE_SEED + 1)
    g, tb = timed(lambda: O.Gamg(A))
    tol, tol_adj = 1e-13, 1e-11
    r, ts = timed(lambda: g.pcg(b, tol=tol, n_pre=1, n_post=1, max_iter=2000))
    assert r.status == O.OK, r.status
    x = r.x
    ra, ta = timed(lambda: g.pcg(x - xt, tol=tol_adj, n_pre=1, n_post=1, max_iter=2000,
                                 transpose=True))
    assert ra.status == O.OK, ra.status
    lam = ra.x
    log(f"c5: forward {r.iterations} it {ts:.1f} s, adjoint {ra.iterations} it {ta:.1f} s")
    gd, gu, gl = O.coeff_grad(A, lam, x)
    # symmetric coefficient c_f: upper = lower = c_f and each end's diagonal
    # loses c_f, so dL/dc_f = g_upper + g_lower - g_diag[own] - g_diag[nb]
    gc = gu + gl - gd[c.owner] - gd[c.neighbour]
    fd_faces = [int(f) for f in c.meta["fd_faces"]]

    # Central differences of L(c_f) at relative step ~1e-6, taken so that
    # rounding in the perturbed system cannot swamp the O(h) change:
    #  - h is the power of two nearest 1e-6 c_f, so c_f +- h and the two
    #    diagonal entries diag -+ h are exact (asserted);
    #  - x(c_f +- h) = x + d+- with A+- d+- = b - A+- x = res -+ h p, where
    #    res = b - A x is formed once (common to both signs, it cancels in
    #    d+ - d-) and p = (x_nb - x_own) e_own + (x_own - x_nb) e_nb is the
    #    exact change of A x per unit h;
    #  - L(c + h) - L(c - h) = (x - x_t).(d+ - d-) + (|d+|^2 - |d-|^2) / 2
    #    exactly, so the two O(|x|^2) losses are never subtracted.
    # Re-assembling the perturbed diagonal instead rounds it by ~eps |diag|,
    # a change whose effect on L (through dL/ddiag = -lambda x, which is far
    # larger than dL/dc_f on smooth fields) reached 1e-4 of dL/dc_f.
    res = b - O.amul(A, x)
    dx = x - xt
    fd, steps = [], []
    for f in fd_faces:
        o, n = int(c.owner[f]), int(c.neighbour[f])
        h = 2.0 ** round(np.log2(1e-6 * c.upper[f]))
        d = []
        for sgn in (1.0, -1.0):
            up = c.upper.copy()
            up[f] += sgn * h
            dg = c.diag.copy()
            dg[o] -= sgn * h
            dg[n] -= sgn * h
            assert up[f] - sgn * h == c.upper[f]
            assert dg[o] + sgn * h == c.diag[o] and dg[n] + sgn * h == c.diag[n]
            rr = res.copy()
            rr[o] -= sgn * h * (x[n] - x[o])
            rr[n] -= sgn * h * (x[o] - x[n])
            ga = O.Gamg(O.Ldu(c.n_cells, c.owner, c.neighbour, dg, up, up))
            s = ga.pcg(rr, tol=1e-12, n_pre=1, n_post=1, max_iter=2000)
            assert s.status == O.OK, s.status
            d.append(s.x)
        dp, dm = d
        v = (dx @ (dp - dm) + 0.5 * (dp @ dp - dm @ dm)) / (2 * h)
        fd.append(float(v))
        steps.append(h / float(c.upper[f]))
        log(f"c5: face {f}: adjoint {gc[f]:.10e} fd {v:.10e} rel {abs(v - gc[f]) / abs(v):.1e}")
    return {"workload": "c5: 100^3 box, 1,000,000 cells, log-normal(0, 0.5) coefficients",
            "sample_seed": SAMPLE_SEED, "indices": idx.tolist(),
            "face_sample_seed": SAMPLE_SEED + 1, "face_indices": fidx.tolist(),
            "tol_forward": tol, "tol_adjoint": tol_adj,
            "forward": solve_record(r, idx, ts),
            "adjoint": solve_record(ra, idx, ta),
            "grad_c_sample": [float(v) for v in gc[fidx]],
            "grad_c_max_abs": float(np.abs(gc).max()),
            "grad_c_norm2": float(np.linalg.norm(gc)),
            "grad_b_norm2": float(np.linalg.norm(lam)),
            "grad_upper_sample": [float(v) for v in gu[fidx]],
            "grad_diag_sample": [float(v) for v in gd[idx]],
            "fd_faces": fd_faces,
            "grad_c_fd_faces": [float(gc[f]) for f in fd_faces],
            "fd_central_rel_step_1e-6": fd, "fd_relative_steps": steps,
            "tol_fd_increments": 1e-12}


def main():
    names = sys.argv[1:] or ["c3", "c4", "c5"]
    for name in names:
        t0 = time.perf_counter()
        out = {"c3": run_c3, "c4": run_c4, "c5": run_c5}[name]()
        out["written_by"] = "tests/golden/make_fullsize_golden.py (oracle only)"
        out["oracle_seconds_total"] = time.perf_counter() - t0
        path = os.path.join(HERE, f"fullsize_{name}.json")
        with open(path, "w") as f:
            json.dump(out, f, separators=(",", ":"))
        log(f"wrote {path}")


if __name__ == "__main__":
    main()
