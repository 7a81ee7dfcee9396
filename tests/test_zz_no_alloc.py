"""pcg_solve_noalloc (the allocation-free entry point) against pcg_solve.

Both run the same kernels in the same launch shapes, so the solution, the
iteration count and the residual history must be bitwise equal; the two
calls in a row (a 32^3 box, then a smaller ragged box) check that the
second call is not disturbed by what the first left in the shared static
scratch.  The free device memory must not change across a call, and calls
outside the entry point's scope are refused.
"""
import ctypes as C

import numpy as np
import pytest

import oracle as O
from meshgen import box_case, config_case, random_order, relabel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _noalloc(m, b, x, hist_len=4096, **kw):
    """One call of pcg_solve_noalloc through the C ABI on caller-owned buffers."""
    from paper_2512_22215_amd import ldu as LL
    L = LL.lib()
    st = LL.Stats()
    buf = (C.c_double * hist_len)()
    st.history = C.cast(buf, C.POINTER(C.c_double))
    st.history_len = hist_len
    o = LL.pcg_opts(**kw)
    rc = L.pcg_solve_noalloc(m._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                             C.byref(o), C.byref(st),
                             C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return rc, st, list(buf[: st.history_count])


def _cases():
    big = config_case("c1")  # 32^3, 32,768 cells
    small = relabel(box_case(21, 17, 13, coeff="lognormal", dirichlet_x0=1.0, seed=11),
                    random_order(21 * 17 * 13, np.random.default_rng(12)))
    return [("c1 32^3", big), ("ragged 21x17x13 random order", small)]


@pytest.mark.parametrize("precond", [1, 0])
def test_noalloc_matches_pcg_solve_two_calls(precond):
    from paper_2512_22215_amd import LduMatrix
    for name, c in _cases():
        print(f"[noalloc] {name}: {c.n_cells} cells, precond {precond}", flush=True)
        m = LduMatrix.from_case(c)
        b = _t(c.rhs[0])
        x_ref, s_ref = m.pcg(b, precond=precond, rel_tol=1e-8, max_iter=5000, history=4096)
        x = torch.zeros_like(b)
        rc, st, hist = _noalloc(m, b, x, precond=precond, rel_tol=1e-8, max_iter=5000)
        assert rc == 0, (rc, m_last_error())
        assert st.iterations == s_ref.iterations and st.converged
        assert torch.equal(x, x_ref), float((x - x_ref).abs().max())
        assert hist == s_ref.history and len(hist) == st.iterations + 1
        assert st.final_residual == s_ref.final_residual
        # against the oracle's solve, at the bars of the existing entry point's
        # parity tests: equal counts, the oracle's residual of x, and for the
        # diagonal preconditioner the solution to 1e-10 (unpreconditioned CG
        # on a lognormal system converges erratically, so two FP64 runs of it
        # part further: solutions within 1e-8 there)
        A = O.Ldu.from_case(c)
        ref = O.pcg(A, c.rhs[0], tol=1e-8, precond=bool(precond))
        assert st.iterations == ref.iterations
        xs = x.cpu().numpy()
        b0 = c.rhs[0]
        assert np.linalg.norm(b0 - O.amul(A, xs)) <= 1e-8 * np.linalg.norm(b0)
        tol = 1e-10 if precond else 1e-8
        assert np.linalg.norm(xs - ref.x) <= tol * np.linalg.norm(ref.x)
        m.close()


def m_last_error():
    from paper_2512_22215_amd import ldu as LL
    return LL.lib().ldu_last_error()


def test_noalloc_allocates_nothing_and_warm_starts():
    from paper_2512_22215_amd import LduMatrix
    c = config_case("c1")
    m = LduMatrix.from_case(c)
    b = _t(c.rhs[0])
    x = torch.zeros_like(b)
    rc, st0, _ = _noalloc(m, b, x, rel_tol=1e-6)  # first call on the device
    assert rc == 0
    free0 = torch.cuda.mem_get_info()[0]
    # a large iteration budget: pcg_solve would size its history buffer from it
    rc, st, _ = _noalloc(m, b, x, rel_tol=1e-10, max_iter=1_000_000)
    free1 = torch.cuda.mem_get_info()[0]
    assert rc == 0 and st.converged
    assert free1 == free0
    # warm start from the 1e-6 iterate: same as pcg_solve from the same x0
    x0 = torch.zeros_like(b)
    _noalloc(m, b, x0, rel_tol=1e-6)
    x_ref, s_ref = m.pcg(b, x0=x0, rel_tol=1e-10, max_iter=1_000_000)
    assert torch.equal(x, x_ref) and st.iterations == s_ref.iterations
    m.close()


def test_noalloc_refuses_out_of_scope_calls():
    from paper_2512_22215_amd import LduMatrix
    from paper_2512_22215_amd.ldu import LDU_ERR_ARG, LDU_ERR_LIMIT
    c = box_case(8, 8, 8, coeff="lognormal", dirichlet_x0=1.0, seed=3)
    m = LduMatrix.from_case(c)
    b = _t(c.rhs[0])
    x = torch.zeros_like(b)
    assert _noalloc(m, b, x, precond=2)[0] == LDU_ERR_ARG
    assert _noalloc(m, b, x, precision="mixed")[0] == LDU_ERR_ARG
    m.close()
    big = box_case(128, 128, 65, coeff="uniform", dirichlet_x0=1.0)  # 1,064,960 cells
    m = LduMatrix.from_case(big)
    b = _t(big.rhs[0])
    x = torch.zeros_like(b)
    assert _noalloc(m, b, x)[0] == LDU_ERR_LIMIT
    assert b"1048576" in m_last_error()
    m.close()
