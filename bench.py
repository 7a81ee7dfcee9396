"""Benchmark: pressure solve to a 1e-8 relative residual on the 8M-cell graded
hex workload (200^3, geometric wall grading, 4 decades of coefficients), and
the achieved HBM bandwidth of the LDU product (Amul) on the same matrix.

One step = one FP64 pressure solve from x0 = 0 to ||b - A x|| / ||b|| <= 1e-8
with CG preconditioned by one GAMG V-cycle per iteration (the hierarchy is set
up once, outside the timed region, as OpenFOAM caches its agglomeration).
Inputs are resident in HBM before timing starts.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--n 200] [--full]

--full also times diagonal PCG, standalone GAMG and the mixed-precision forms
(minutes); the default run finishes in about two minutes.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pressure-solve time to 1e-8 rel. residual at 8M cells; Amul HBM GB/s"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
# GAMG hierarchies of the headline solve: pairwise handshake matching on
# every level (the paper's GAMG default), or pairwise from level 0 to 1 and
# three matching passes per level below, aggregates of about eight cells
# (the aggressive coarsening the paper names as the remedy for GAMG's many
# small levels on GPUs, Sec. 4.4)
HIERARCHIES = {"pairwise": {}, "aggressive": {"passes": 3, "aggressive_from": 1}}
AGG_TEXT = {"pairwise": "pairwise agglomeration on every level",
            "aggressive": "pairwise agglomeration from level 0 to 1, three matching passes "
                          "per level below"}


def measured_traffic():
    """Calibrated HBM bytes per Amul launch from the committed counter runs, or
    None when the kernel sources changed after the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "amul_c3_counters.json")
    try:
        rec = json.load(open(path))
        src = b"".join(open(os.path.join(ROOT, f), "rb").read() for f in rec["source_files"])
        if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
            return None
        return rec["amul_f64"]["traffic_bytes"]
    except (OSError, KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def amul_bytes(n, nf):
    """Algorithmic bytes of one FP64 Amul: diag, x, y (8 B each per cell) and
    upper, lower (8 B each) plus owner/neighbour addressing (4 B each) per face.
    The coefficient gradient moves the same count: lambda, x, g_diag per cell;
    owner, neighbour, g_upper, g_lower per face."""
    return 24 * n + 24 * nf


def time_kernel(fn, reps, torch):
    """Average duration of fn() over reps back-to-back launches, measured with
    HIP events on the stream the library launches on (torch's current)."""
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def host_cpu():
    """(threads the process may use, CPU model) of the host."""
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count()
    model = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return cores, model


def cpu_baseline(case, iters_gpu, sweeps, t_gpu, sample_iters=6, hierarchy=None):
    """The serial oracle on the host, on the full workload (the same matrix
    and right-hand side as the GPU step), timed in pieces that keep the run
    bounded: its Amul (mean of 5 calls), its GAMG build with the same
    agglomeration settings (reported, not counted), and sample_iters
    iterations of the same V-cycle-preconditioned CG (sweeps + sweeps Jacobi
    sweeps).  The per-iteration time times the
    GPU's iteration count estimates one oracle solve; COE (Sec. 4.3,
    coefficient of equivalence) = T_cpu * N_cores / (T_gpu * N_gpus) with
    one core and one GPU."""
    import oracle as O
    A = O.Ldu.from_case(case)
    x = np.random.default_rng(7).standard_normal(case.n_cells)
    ta = []
    for _ in range(5):
        t0 = time.perf_counter()
        O.amul(A, x)
        ta.append(time.perf_counter() - t0)
    t_amul = float(np.mean(ta))
    t0 = time.perf_counter()
    g = O.Gamg(A, **(hierarchy or {}))
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    r = g.pcg(case.rhs[0], tol=1e-8, max_iter=sample_iters, n_pre=sweeps, n_post=sweeps)
    t_iter = (time.perf_counter() - t0) / max(r.iterations, 1)
    cores, model = host_cpu()
    value = t_iter * iters_gpu
    return {
        "value": value,
        "unit": "s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"serial C oracle, 1 thread of {model} (host exposes {cores}), measured at "
                   f"{case.n_cells:,} cells on the same matrix and rhs: {r.iterations} CG "
                   f"iterations with one {sweeps}+{sweeps}-sweep V-cycle each at {t_iter:.3f} s "
                   f"per iteration ({g.n_levels} levels, agglomeration {hierarchy or 'pairwise'}), "
                   f"times the GPU's {iters_gpu} iterations; GAMG build {t_build:.1f} s not "
                   f"counted"),
        "oracle_amul_s": t_amul,
        "oracle_amul_GBps": amul_bytes(case.n_cells, case.n_faces) / t_amul / 1e9,
        "oracle_gamg_build_s": t_build,
        "oracle_s_per_iteration": t_iter,
        "coe_vs_serial_oracle": value / t_gpu,
    }


def stream_ceilings(torch, dev, n_cells):
    """Hand-written HBM stream kernels (include/ldu_bench.h) timed with HIP
    events on the current stream, each the best over grid sizes and over
    plain and nontemporal accesses: a read-only sum and a copy of 1 GiB
    arrays (well above the 256 MB Infinity Cache), and the CG's x/r update
    over n_cells cells (at 8M cells its four vectors, 256 MB, partly stay in
    that cache)."""
    import ctypes as C

    from paper_2512_22215_amd import lib
    L = lib()
    st = lambda: C.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda t: C.c_void_p(t.data_ptr())

    def best(fn, nbytes):
        runs = {}
        for nt in (0, 1):
            for blocks in (1024, 2048, 4096, 8192):
                t = time_kernel(lambda: fn(blocks, nt), 20, torch)
                runs[(blocks, nt)] = t
        (blocks, nt), t = min(runs.items(), key=lambda kv: kv[1])
        plain = min(v for (bl, n_), v in runs.items() if n_ == 0)
        return {"GBps": nbytes / t / 1e9, "bytes": nbytes, "blocks": blocks,
                "nontemporal": bool(nt), "GBps_plain": nbytes / plain / 1e9}

    out = {}
    nread = 2 * 64 * 1024 * 1024  # 1 GiB of doubles, well above the caches
    a = torch.rand(nread, dtype=torch.float64, device=dev)
    part = torch.empty(8192, dtype=torch.float64, device=dev)
    out["read"] = best(lambda bl, nt: L.ldu_stream_read(p(a), nread, p(part), bl, nt, st()),
                       8 * nread)
    b = torch.empty_like(a)
    out["copy"] = best(lambda bl, nt: L.ldu_stream_copy(p(a), p(b), nread, bl, nt, st()),
                       16 * nread)
    del a, b
    vs = [torch.rand(n_cells, dtype=torch.float64, device=dev) for _ in range(4)]
    out["cg_update"] = best(
        lambda bl, nt: L.ldu_stream_cg_update(p(vs[0]), p(vs[1]), p(vs[2]), p(vs[3]),
                                              C.c_double(1e-3), n_cells, bl, nt, st()),
        48 * n_cells)
    out["cg_update"]["cells"] = n_cells
    del vs
    torch.cuda.synchronize()
    return out


def load_golden(name):
    """The oracle's full-size reference results (tests/golden, written by a
    script that calls only the oracle), or None."""
    path = os.path.join(ROOT, "tests", "golden", f"fullsize_{name}.json")
    try:
        return json.load(open(path))
    except (OSError, ValueError):
        return None


def sampled_error(x, gold, rec):
    """||x - x_orc|| / ||x_orc|| over the oracle's sampled cells, and the
    relative difference of the 2-norms of the whole vectors (x: a device
    tensor)."""
    if gold is None or rec is None:
        return None
    import torch
    idx = np.asarray(gold["indices"], dtype=np.int64)
    want = np.asarray(rec["x"]["sample"])
    got = x[torch.from_numpy(idx).to(x.device)].cpu().numpy()
    return {"sampled_rel_err": float(np.linalg.norm(got - want) / np.linalg.norm(want)),
            "norm2_rel_diff": float(abs(float(x.norm()) - rec["x"]["norm2"]) /
                                    rec["x"]["norm2"]),
            "samples": int(idx.size), "oracle_iterations": rec["iterations"]}


def _timed(torch, fn, reps=2):
    """One warm-up call, then the best of reps timed calls (seconds)."""
    out = fn()
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best, out


def run_suite(torch, dev, only=None):
    """The runs each workload is defined for, timed on the GPU: c1 PCG; c2
    PCG, GAMG and CG + V-cycle in random and RCM numbering; c4 PCG FP64 and
    mixed over three warm-started right-hand sides, plus CG + V-cycle; c5
    forward and adjoint with the coefficient gradients.  Every solve is checked
    against its tolerance through the library's FP64 residual."""
    from meshgen import config_case
    from paper_2512_22215_amd import LduMatrix

    def tens(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    def solve_rec(m, b, fn, **kw):
        t, (x, st) = _timed(torch, lambda: fn(b, **kw))
        res = m.residual(b, x)
        assert st.converged and res <= kw.get("rel_tol", 1e-8) * 1.0000001, (kw, st, res)
        return {"s": t, "iterations": st.iterations, "refinements": st.refinements,
                "true_residual": res}

    def amul_rec(m, case):
        x = torch.randn(case.n_cells, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        t = time_kernel(lambda: m.amul(x, out=y), 100, torch)
        return {"us": t * 1e6, "GBps": amul_bytes(case.n_cells, case.n_faces) / t / 1e9}

    import oracle as O
    cores, model = host_cpu()
    host = f"serial C oracle, 1 thread of {model} (host exposes {cores})"

    def oracle_amul(case):
        A = O.Ldu.from_case(case)
        x = np.random.default_rng(7).standard_normal(case.n_cells)
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            O.amul(A, x)
            ts.append(time.perf_counter() - t0)
        t = float(np.mean(ts))
        return {"s": t, "GBps": amul_bytes(case.n_cells, case.n_faces) / t / 1e9, "host": host}

    def oracle_solve(label, fn, t_gpu):
        t0 = time.perf_counter()
        r = fn()
        t = time.perf_counter() - t0
        return {"solver": label, "s": t, "iterations": r.iterations, "status": r.status,
                "host": host, "coe_vs_serial_oracle": t / t_gpu}

    for name, kw in (("c1", {}), ("c2", {"order": "random"}), ("c2", {"order": "rcm"}),
                     ("c4", {}), ("c5", {})):
        label = name + ("-rcm" if kw.get("order") == "rcm" else "")
        if only and label != only:
            continue
        t0 = time.perf_counter()
        case = config_case(name, **kw)
        log(f"[suite] {case.name}: {case.n_cells} cells ({time.perf_counter() - t0:.1f} s "
            f"to generate)")
        m = LduMatrix.from_case(case)
        rec = {"workload": case.name, "cells": case.n_cells, "faces": case.n_faces,
               "amul_f64": amul_rec(m, case)}
        b = tens(case.rhs[0])
        if name in ("c2", "c4"):
            rec["oracle_amul_f64"] = oracle_amul(case)
        if name == "c1":
            rec["pcg_diag_fp64"] = solve_rec(m, b, m.pcg, rel_tol=1e-8)
            A = O.Ldu.from_case(case)
            rec["oracle_pcg_diag_fp64"] = oracle_solve(
                "diagonal PCG, FP64, 1e-8", lambda: O.pcg(A, case.rhs[0], tol=1e-8),
                rec["pcg_diag_fp64"]["s"])
        elif name == "c2":
            rec["pcg_diag_fp64"] = solve_rec(m, b, m.pcg, rel_tol=1e-8)
            m.gamg_setup(n_pre=1, n_post=1)
            rec["levels"] = m.n_levels()
            rec["gamg_fp64"] = solve_rec(m, b, m.gamg, rel_tol=1e-8, n_pre=1, n_post=1,
                                         max_cycles=1000)
            rec["pcg_gamg_fp64"] = solve_rec(m, b, m.pcg, rel_tol=1e-8, precond=2)
        elif name == "c4":
            # stream ceilings timed in the same run, the CG update at this size
            # (its vectors, 134 MB each, do not fit the Infinity Cache)
            rec["ceilings"] = stream_ceilings(torch, dev, case.n_cells)
            m.gamg_setup(n_pre=1, n_post=1)
            rec["levels"] = m.n_levels()
            gold = load_golden("c4")
            for label, kwp in (("pcg_diag", dict(rel_tol=1e-8)),
                               ("pcg_gamg", dict(rel_tol=1e-8, precond=2))):
                for prec in ("fp64", "mixed"):
                    runs = []
                    xk = torch.zeros(case.n_cells, dtype=torch.float64, device=dev)
                    for k, rk in enumerate(case.rhs):  # back to back, each warm-started
                        bk = tens(rk)
                        torch.cuda.synchronize()
                        t1 = time.perf_counter()
                        xk, st = m.pcg(bk, x0=xk, precision=prec, **kwp)
                        torch.cuda.synchronize()
                        dt = time.perf_counter() - t1
                        res = m.residual(bk, xk)
                        assert st.converged and res <= 1e-8, (label, prec, st, res)
                        # error against the oracle's FP64 solve of the same rhs
                        orec = gold[f"{label}_fp64"][k] if gold else None
                        runs.append({"s": dt, "iterations": st.iterations,
                                     "refinements": st.refinements, "true_residual": res,
                                     "vs_fp64_oracle": sampled_error(xk, gold, orec)})
                    rec[f"{label}_{prec}_3rhs"] = runs
        elif name == "c5":
            rec["pcg_diag_fp64"] = solve_rec(m, b, m.pcg, rel_tol=1e-8)
            rec["pcg_diag_mixed"] = solve_rec(m, b, m.pcg, rel_tol=1e-8, precision="mixed")
            m.gamg_setup(n_pre=1, n_post=1)
            rec["pcg_gamg_fp64"] = solve_rec(m, b, m.pcg, rel_tol=1e-8, precond=2)
            rec["pcg_gamg_mixed"] = solve_rec(m, b, m.pcg, rel_tol=1e-8, precond=2,
                                              precision="mixed")
            A = O.Ldu.from_case(case)
            g = O.Gamg(A)
            rec["oracle_pcg_gamg_fp64"] = oracle_solve(
                "CG + V-cycle (1+1), FP64, 1e-8",
                lambda: g.pcg(case.rhs[0], tol=1e-8, n_pre=1, n_post=1),
                rec["pcg_gamg_fp64"]["s"])
            del g
            # the differentiable solve: loss = |x - x_t|^2 / 2 through LduSolve,
            # gradients for every symmetric face coefficient and b, forward +
            # backward, FP64 and FP32-bulk-with-FP64-refinement, both to 1e-11
            from paper_2512_22215_amd import ldu_solve
            own = torch.from_numpy(case.owner.astype(np.int64)).to(dev)
            nbi = torch.from_numpy(case.neighbour.astype(np.int64)).to(dev)
            ab = tens(case.meta["a_boundary"])
            xt = tens(case.meta["x_target"])
            zero = torch.zeros(case.n_cells, dtype=torch.float64, device=dev)
            grads = {}
            gold = load_golden("c5")
            errs = {}
            for prec in ("fp64", "mixed", "fp64", "mixed"):  # the first pair warms up
                a = tens(case.upper).requires_grad_(True)
                bb = tens(case.rhs[0]).requires_grad_(True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                d = -(zero.index_add(0, own, a).index_add(0, nbi, a)) - ab
                x = ldu_solve(d, a, a, bb, m, "pcg", precond=2, precision=prec, rel_tol=1e-11)
                (0.5 * torch.sum((x - xt) ** 2)).backward()
                torch.cuda.synchronize()
                grads[prec] = (time.perf_counter() - t0, a.grad)
                if gold:  # against the oracle's full-size adjoint run (sampled)
                    fidx = torch.from_numpy(np.asarray(gold["face_indices"])).to(dev)
                    cidx = torch.from_numpy(np.asarray(gold["indices"])).to(dev)

                    def rel(got, idx, want):
                        want = np.asarray(want)
                        got = got.detach()[idx].cpu().numpy()
                        return float(np.linalg.norm(got - want) / np.linalg.norm(want))
                    fd = np.asarray(gold["fd_central_rel_step_1e-6"])
                    gfd = a.grad[torch.from_numpy(np.asarray(gold["fd_faces"])).to(dev)]
                    errs[prec] = {
                        "x": rel(x, cidx, gold["forward"]["x"]["sample"]),
                        "dL_db": rel(bb.grad, cidx, gold["adjoint"]["x"]["sample"]),
                        "dL_dc": rel(a.grad, fidx, gold["grad_c_sample"]),
                        "fd_max_rel": float(np.max(np.abs(gfd.cpu().numpy() - fd) /
                                                   np.abs(fd)))}
            rec["autograd_forward_backward_1e-11"] = {
                "fp64_s": grads["fp64"][0], "mixed_s": grads["mixed"][0],
                "grad_mixed_vs_fp64_rel": float(torch.linalg.norm(grads["mixed"][1] -
                                                                  grads["fp64"][1]) /
                                                torch.linalg.norm(grads["fp64"][1])),
                "vs_oracle": errs or None}
            lam = tens(np.zeros(case.n_cells))
            tg = time_kernel(lambda: m.coeff_grad(lam, zero), 20, torch)
            rec["coeff_grad_us"] = tg * 1e6
        m.close()
        log(f"[suite] {json.dumps(rec)}")
        print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=200)
    ap.add_argument("--full", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--sweeps", type=int, default=1,
                    help="Jacobi sweeps before and after the coarse correction")
    ap.add_argument("--agglomeration", choices=("aggressive", "pairwise"), default="aggressive",
                    help="hierarchy of the timed solve: pairwise matching from level 0 to 1 "
                         "and three matching passes per level below (aggressive), or "
                         "pairwise matching on every level")
    ap.add_argument("--amul-only", action="store_true",
                    help="only the Amul and copy timings (for counter runs)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the mixed, adjoint and variant solves (for kernel traces)")
    ap.add_argument("--suite", action="store_true",
                    help="instead of the headline step, time the runs of every workload "
                         "(c1, c2 random and RCM, c4, c5), one JSON line each")
    ap.add_argument("--only", default=None,
                    help="with --suite: run one workload (c1, c2, c2-rcm, c4, c5)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1 "
                          "(sharding over several GPUs is not implemented)"}))
        sys.exit(2)

    import torch

    from meshgen import config_case
    from paper_2512_22215_amd import LduMatrix

    dev = torch.device("cuda:0")
    if args.suite:
        run_suite(torch, dev, args.only)
        return
    t0 = time.perf_counter()
    case = config_case("c3", n=args.n)
    log(f"[bench] workload c3 n={args.n}: {case.n_cells} cells, {case.n_faces} faces "
        f"({time.perf_counter() - t0:.1f} s to generate)")
    own = torch.from_numpy(case.owner).to(dev)
    nb = torch.from_numpy(case.neighbour).to(dev)
    d = torch.from_numpy(case.diag).to(dev)
    up = torch.from_numpy(case.upper).to(dev)
    lo = torch.from_numpy(case.lower).to(dev)
    b = torch.from_numpy(case.rhs[0]).to(dev)
    torch.cuda.synchronize()

    # device memory the library holds (free HBM before and after; the inputs
    # above are the caller's and already allocated)
    free0 = torch.cuda.mem_get_info(dev)[0]
    t0 = time.perf_counter()
    m = LduMatrix(case.n_cells, own, nb, d, up, lo, device=dev)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    free1 = torch.cuda.mem_get_info(dev)[0]
    hier = HIERARCHIES[args.agglomeration]
    t0 = time.perf_counter()
    m.gamg_setup(n_pre=args.sweeps, n_post=args.sweeps, **hier)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    free2 = torch.cuda.mem_get_info(dev)[0]
    mem = {"level0_bytes": free0 - free1, "hierarchy_bytes": free1 - free2}
    nlev = m.n_levels()
    log(f"[bench] ldu_create {t_create:.3f} s, gamg_setup {t_setup:.3f} s, {nlev} levels")

    # ---- Amul roofline (the dominant kernel family of every solver here)
    x = torch.randn(case.n_cells, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    t_amul = time_kernel(lambda: m.amul(x, out=y), 200, torch)
    abytes = amul_bytes(case.n_cells, case.n_faces)
    amul_gbs = abytes / t_amul / 1e9
    log(f"[bench] Amul {t_amul * 1e6:.1f} us, {amul_gbs:.0f} GB/s algorithmic")
    x32 = x.float()
    y32 = torch.empty_like(x32)
    t_amul32 = time_kernel(lambda: m.amul_f32(x32, out=y32), 200, torch)
    a32bytes = 12 * case.n_cells + 16 * case.n_faces
    # HBM ceilings of hand-written stream kernels, timed in this run
    ceil = stream_ceilings(torch, dev, case.n_cells)
    copy_gbs = ceil["copy"]["GBps"]
    log(f"[bench] ceilings: read {ceil['read']['GBps']:.0f}, copy {copy_gbs:.0f}, "
        f"CG update {ceil['cg_update']['GBps']:.0f} GB/s")
    if args.amul_only:
        print(json.dumps({"amul_us": t_amul * 1e6, "amul_GBps": amul_gbs,
                          "amul_bytes": abytes, "ceilings": ceil}))
        m.close()
        return

    # ---- the timed steps: pressure solves
    opts = dict(precond=2, rel_tol=1e-8, max_iter=2000)
    for _ in range(args.warmup):
        xs, st = m.pcg(b, **opts)
    torch.cuda.synchronize()
    times = []
    for k in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xs, st = m.pcg(b, **opts)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log(f"[bench] step {k}: {times[-1]:.4f} s, {st.iterations} iterations, "
            f"final residual {st.final_residual:.3e}")
    res = m.residual(b, xs)
    assert st.converged and res <= 1e-8, (st, res)
    t_step = float(np.mean(times))
    gold = load_golden("c3") if args.n == 200 else None
    gkey = "pcg_gamg_fp64" + ("_aggressive" if args.agglomeration == "aggressive" else "")
    grec = gold.get(gkey) if gold else None
    err64 = sampled_error(xs, gold, grec)
    if err64:
        log(f"[bench] FP64 vs oracle: sampled |x - x_orc|/|x_orc| "
            f"{err64['sampled_rel_err']:.2e}, oracle {grec['iterations']} iterations")

    variants, mixed_rec, adj_rec, bicg_rec, gamg_rec = {}, None, None, None, None
    if not args.no_extra:
        # the mixed form of the same solve: FP64 refinement around FP32 CG with an
        # FP32 V-cycle preconditioner (one warm-up, then the same step count)
        mopts = dict(opts, precision="mixed")
        m.pcg(b, **mopts)
        mtimes = []
        for k in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xm, sm = m.pcg(b, **mopts)
            torch.cuda.synchronize()
            mtimes.append(time.perf_counter() - t0)
        mres = m.residual(b, xm)
        assert sm.converged and mres <= 1e-8, (sm, mres)
        log(f"[bench] mixed: {np.mean(mtimes):.4f} s, {sm.refinements} refinements, "
            f"{sm.iterations} inner iterations, true residual {mres:.3e}")
        mixed_rec = {"s": float(np.mean(mtimes)), "refinements": sm.refinements,
                     "inner_iterations": sm.iterations, "true_residual": mres,
                     "solver": "FP64 refinement, FP32 CG + FP32 V-cycle (FP64 coarsest)",
                     "vs_fp64_oracle": sampled_error(xm, gold, grec)}

        # standalone GAMG (x += V(b - A x) per cycle, correction scaling on)
        # from x0 = 0 with a 400-cycle cap, FP64 and mixed, on the headline
        # hierarchy: the configured c3 solver; its convergence factor per cycle
        # is what makes CG + V-cycle the headline solver on this graded mesh
        gamg_rec = {}
        for label, kw in (("fp64_1+1", dict(n_pre=args.sweeps, n_post=args.sweeps)),
                          ("fp64_2+2", dict(n_pre=2, n_post=2)),
                          ("mixed_1+1", dict(n_pre=args.sweeps, n_post=args.sweeps,
                                             precision="mixed", max_refine=400))):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xg, sg = m.gamg(b, rel_tol=1e-8, max_cycles=400, history=500, **hier, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            h = np.asarray(sg.history)
            k = len(h) - 1
            gamg_rec[label] = {
                "s": dt, "cycles": sg.refinements if kw.get("precision") else sg.iterations,
                "converged": sg.converged, "final_residual": sg.final_residual,
                "factor_per_cycle": float((h[-1] / h[0]) ** (1.0 / k)) if k > 0 else None,
                "factor_last_20": float((h[-1] / h[-21]) ** (1.0 / 20)) if k > 20 else None,
                "cycles_to_1e-8_at_that_rate": (
                    float(np.log(1e-8 / h[-1]) / np.log((h[-1] / h[-21]) ** (1.0 / 20)) + k)
                    if k > 20 and h[-1] > 1e-8 else None)}
            log(f"[bench] standalone GAMG {label}: {dt:.3f} s, {gamg_rec[label]}")

        # the adjoint form: lambda = A^-T (x - x_t) with the same preconditioned CG
        # (on the transposed values of every level), then the per-face gradients
        xt = torch.randn(case.n_cells, dtype=torch.float64, device=dev,
                         generator=torch.Generator(device=dev).manual_seed(4))
        g = xs - xt
        m.adjoint(g, **opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam, sa = m.adjoint(g, **opts)
        torch.cuda.synchronize()
        t_adj = time.perf_counter() - t0
        gd, gu, gl = m.coeff_grad(lam, xs)
        t_grad = time_kernel(lambda: m.coeff_grad(lam, xs), 20, torch)
        assert sa.converged
        log(f"[bench] adjoint: {t_adj:.4f} s, {sa.iterations} iterations; coeff_grad "
            f"{t_grad * 1e6:.0f} us")
        adj_rec = {"solve_s": t_adj, "iterations": sa.iterations,
                   "coeff_grad_us": t_grad * 1e6,
                   "coeff_grad_GBps": amul_bytes(case.n_cells, case.n_faces) / t_grad / 1e9}

        def timed_pcg(vo, reps=2):
            m.pcg(b, **vo)
            vt = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                xv, sv = m.pcg(b, **vo)
                torch.cuda.synchronize()
                vt.append(time.perf_counter() - t0)
            vres = m.residual(b, xv)
            assert sv.converged and vres <= 1e-8, (vo, sv, vres)
            return xv, {"s": float(np.mean(vt)), "iterations": sv.iterations,
                        "refinements": sv.refinements, "true_residual": vres}

        variants = {}
        # the other hierarchy of the headline solve, timed as the headline is
        # (warm-up, then the mean of `steps` solves), against its oracle run
        other = "pairwise" if args.agglomeration == "aggressive" else "aggressive"
        m.gamg_setup(n_pre=args.sweeps, n_post=args.sweeps, **HIERARCHIES[other])
        okey = "pcg_gamg_fp64" + ("_aggressive" if other == "aggressive" else "")
        rec = {"levels": m.n_levels(), "settings": HIERARCHIES[other]}
        for prec in ("fp64", "mixed"):
            xv, rec[prec] = timed_pcg(dict(opts, precision=prec), reps=args.steps)
            orec = gold.get(okey) if gold else None
            rec[prec]["vs_fp64_oracle"] = sampled_error(xv, gold, orec)
        variants[other + "_hierarchy"] = rec
        log(f"[bench] {other} hierarchy: {rec['levels']} levels, fp64 {rec['fp64']['s']:.4f} s "
            f"({rec['fp64']['iterations']} it), mixed {rec['mixed']['s']:.4f} s")

        # agglomeration settings: pairwise matching down to level `from`, then
        # 2 or 3 matching passes per level (FP64 and mixed, warm-up + mean of 2)
        sweep = {}
        for afrom, passes in ((0, 2), (0, 3), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3), (4, 3),
                              (6, 3)):
            m.gamg_setup(n_pre=args.sweeps, n_post=args.sweeps, passes=passes,
                         aggressive_from=afrom)
            r = {"levels": m.n_levels()}
            for prec in ("fp64", "mixed"):
                r[prec] = timed_pcg(dict(opts, precision=prec))[1]
            sweep[f"from{afrom}_passes{passes}"] = r
        best = min(sweep, key=lambda k: sweep[k]["fp64"]["s"])
        variants["agglomeration_sweep"] = {"runs": sweep, "best_fp64": best}
        log(f"[bench] agglomeration sweep: best {best} {sweep[best]}")

        # the two-stage Gauss-Seidel smoother and the DIC coarsest
        # preconditioner on the headline hierarchy
        for name, kw in (("gs2_smoother", dict(smoother="gs2")),
                         ("dic_coarsest", dict(coarsest="dic"))):
            t0 = time.perf_counter()
            m.gamg_setup(n_pre=args.sweeps, n_post=args.sweeps, **hier, **kw)
            torch.cuda.synchronize()
            rec = {"setup_s": time.perf_counter() - t0, "levels": m.n_levels()}
            for prec in ("fp64", "mixed"):
                rec[prec] = timed_pcg(dict(opts, precision=prec))[1]
            variants[name] = rec
            log(f"[bench] variant {name}: {rec['levels']} levels, fp64 {rec['fp64']['s']:.4f} s "
                f"({rec['fp64']['iterations']} it), mixed {rec['mixed']['s']:.4f} s")
        m.gamg_setup(n_pre=args.sweeps, n_post=args.sweeps, **hier)

        # the non-symmetric solve (PBiCG, diagonal preconditioner) on the
        # convection-diffusion box of the same size (200^3, upwind, Courant 2)
        cu = config_case("c5u", n=args.n)
        mu = LduMatrix.from_case(cu)
        bu = torch.from_numpy(cu.rhs[0]).to(dev)
        mu.pbicg(bu, rel_tol=1e-8, max_iter=5000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xu, su = mu.pbicg(bu, rel_tol=1e-8, max_iter=5000)
        torch.cuda.synchronize()
        t_bicg = time.perf_counter() - t0
        ures = mu.residual(bu, xu)
        assert su.converged and ures <= 1e-8, (su, ures)
        log(f"[bench] PBiCG on the {args.n}^3 convection-diffusion box: {t_bicg:.4f} s, "
            f"{su.iterations} iterations")
        bicg_rec = {"s": t_bicg, "iterations": su.iterations, "true_residual": ures,
                    "workload": f"c5u: {args.n}^3 upwind convection-diffusion, {cu.n_cells} cells",
                    "ms_per_iteration": t_bicg / max(su.iterations, 1) * 1e3}
        mu.close()
        del mu, xu, bu

        # pressure-equation assembly from geometry on the same mesh (face
        # interpolation, Laplacian, negSumDiag, divergence) including the
        # refresh of a cached GAMG hierarchy's Galerkin values
        from meshgen import c3_assembly_inputs
        ga = c3_assembly_inputs(n=args.n)
        nfa = ga["owner"].size
        ma = LduMatrix(ga["n"], torch.from_numpy(ga["owner"].astype(np.int32)).to(dev),
                       torch.from_numpy(ga["neighbour"].astype(np.int32)).to(dev),
                       torch.full((ga["n"],), -6.0, dtype=torch.float64, device=dev),
                       torch.ones(nfa, dtype=torch.float64, device=dev),
                       torch.ones(nfa, dtype=torch.float64, device=dev), device=dev)
        aargs = [torch.from_numpy(ga[k]).to(dev) for k in ("gamma", "weights", "mag_sf", "delta")]
        akw = {k: torch.from_numpy(ga[k]).to(dev) for k in ("diag_bc", "phi", "b_bc")}
        asm = {}
        for label, refresh in (("assemble", False), ("assemble_and_refresh_gamg", True)):
            if refresh:
                ma.gamg_setup(n_pre=args.sweeps, n_post=args.sweeps,
                              **HIERARCHIES[args.agglomeration])
            ma.assemble_pressure(*aargs, **akw)
            at = []
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ma.assemble_pressure(*aargs, **akw)
                torch.cuda.synchronize()
                at.append(time.perf_counter() - t0)
            asm[label + "_ms"] = float(np.min(at)) * 1e3
        log(f"[bench] pressure assembly {asm['assemble_ms']:.2f} ms, with GAMG refresh "
            f"{asm['assemble_and_refresh_gamg_ms']:.2f} ms")
        ma.close()
        del ma, aargs, akw

    extra = {
        "pressure_assembly": asm if not args.no_extra else None,
        "pbicg_nonsymmetric": bicg_rec,
        "variants": variants,
        "adjoint": adj_rec,
        "mixed_solve": mixed_rec,
        "setup_s": {"ldu_create": t_create, "gamg_setup": t_setup},
        "device_memory": mem,
        "levels": nlev,
        "iterations": st.iterations,
        "true_residual": res,
        "amul_f64": {"us": t_amul * 1e6, "GBps": amul_gbs, "bytes": abytes},
        "amul_f32": {"us": t_amul32 * 1e6, "GBps": a32bytes / t_amul32 / 1e9,
                     "bytes": a32bytes},
        "ceilings": ceil,
        # Amul moves ~90% reads: its algorithmic rate against the read ceiling
        "amul_frac_of_read_ceiling": amul_gbs / ceil["read"]["GBps"],
        "fp64_vs_oracle": err64,
        "standalone_gamg": gamg_rec if not args.no_extra else None,
    }
    if args.full:
        for name, fn, kw in (
                ("pcg_diag_fp64", m.pcg, dict(rel_tol=1e-8, max_iter=50000)),
                ("pcg_diag_mixed", m.pcg, dict(rel_tol=1e-8, precision="mixed")),
                ("gamg_fp64", m.gamg, dict(rel_tol=1e-8, max_cycles=3000)),
                ("gamg_mixed", m.gamg, dict(rel_tol=1e-8, precision="mixed",
                                            max_refine=3000))):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xo, so = fn(b, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            extra[name] = {"s": dt, "iterations": so.iterations,
                           "refinements": so.refinements, "converged": so.converged,
                           "true_residual": m.residual(b, xo)}
            log(f"[bench] {name}: {dt:.3f} s {so.iterations} it conv={so.converged}")

    out = {
        "metric": METRIC,
        "value": t_step,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"c3: {args.n}^3 graded hex, {case.n_cells} cells, "
                               f"{case.n_faces} faces, Dirichlet top, N(0,1) rhs",
                   "solver": f"CG + GAMG V-cycle ({AGG_TEXT[args.agglomeration]}, "
                             f"{nlev} levels, {args.sweeps}+{args.sweeps} Jacobi sweeps "
                             f"w=0.75, diagonal-CG coarsest)",
                   "rel_tol": 1e-8, "x0": "zero"},
        "roofline": {"bound": "hbm", "kernel": "ldu_amul (k_amul<double>)",
                     "achieved": amul_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": amul_gbs / HBM_PEAK_GBS,
                     "traffic": measured_traffic() if args.n == 200 else None},
        "extra": extra,
    }
    if not args.no_cpu:
        log("[bench] timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(case, st.iterations, args.sweeps, t_step,
                                           hierarchy=hier)
        log(f"[bench] oracle estimate {out['cpu_baseline']['value']:.1f} s per solve")
    m.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
