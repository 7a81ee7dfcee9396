"""Box meshes in OpenFOAM LDU form (face addressing with owner < neighbour).

The paper keeps OpenFOAM's lduMatrix storage, where the sparsity pattern is the
mesh face graph (Sec. 2.1, "Design aspects"): a diagonal per cell plus one
upper and one lower coefficient per internal face, addressed by the face's
owner and neighbour cell.  Convention used throughout: A[owner, neighbour] =
upper, A[neighbour, owner] = lower, faces sorted by (owner, neighbour).

The five workloads below stand in for the paper's DrivAer meshes (Sec. 4.1),
which are not available: boxes with 2.9-3.0 internal faces per cell, an
unstructured (randomly permuted) numbering, wall grading with four decades of
coefficient spread, and a 16.7M-cell case above the paper's "more than 10M
cells per GPU" load.  Every random draw uses numpy's default_rng(1000*c + s)
with s = 1 permutation, 2 coefficient noise, 3 rhs, 4 adjoint target, 5 face
pick, so each case is reproducible bit for bit.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

CONFIG_NAMES = ("c1", "c2", "c3", "c4", "c5")


@dataclass
class LduCase:
    """One linear system A x = b in LDU form plus case metadata."""

    name: str
    n_cells: int
    owner: np.ndarray  # int32 [F]
    neighbour: np.ndarray  # int32 [F]
    diag: np.ndarray  # float64 [N]
    upper: np.ndarray  # float64 [F]
    lower: np.ndarray  # float64 [F]
    rhs: list = field(default_factory=list)  # list of float64 [N]
    singular: bool = False  # pure zero-gradient (constant null space)
    meta: dict = field(default_factory=dict)

    @property
    def n_faces(self) -> int:
        return int(self.owner.shape[0])


def box_faces(nx: int, ny: int, nz: int):
    """Internal faces of an nx*ny*nz box with cell index i = ix + nx*(iy + ny*iz).

    Returns (owner, neighbour, axis) sorted by (owner, neighbour); axis is 0/1/2
    for x/y/z faces.  The count is (nx-1)ny nz + nx(ny-1)nz + nx ny(nz-1).
    """
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64).reshape(nz, ny, nx)
    own = []
    nb = []
    ax = []
    if nx > 1:
        o = idx[:, :, :-1].ravel()
        own.append(o)
        nb.append(o + 1)
        ax.append(np.zeros(o.size, np.int8))
    if ny > 1:
        o = idx[:, :-1, :].ravel()
        own.append(o)
        nb.append(o + nx)
        ax.append(np.ones(o.size, np.int8))
    if nz > 1:
        o = idx[:-1, :, :].ravel()
        own.append(o)
        nb.append(o + nx * ny)
        ax.append(np.full(o.size, 2, np.int8))
    if not own:
        z = np.zeros(0, np.int32)
        return z, z.copy(), np.zeros(0, np.int8)
    own = np.concatenate(own)
    nb = np.concatenate(nb)
    ax = np.concatenate(ax)
    order = np.lexsort((nb, own))
    return (own[order].astype(np.int32), nb[order].astype(np.int32),
            ax[order])


def assemble_diag(n: int, owner, neighbour, upper, lower, a_boundary=None):
    """diag_i = -(sum of the off-diagonal entries of row i) - a_boundary_i.

    Row i of the LDU matrix holds upper_f for faces it owns and lower_f for
    faces where it is the neighbour, so a pure zero-gradient system has zero
    row sums; a Dirichlet boundary adds a positive coefficient a_b to -diag.
    """
    d = -(np.bincount(owner, weights=upper, minlength=n)
          + np.bincount(neighbour, weights=lower, minlength=n))
    if a_boundary is not None:
        d = d - a_boundary
    return d.astype(np.float64)


def relabel(case: LduCase, newidx: np.ndarray, name: str | None = None):
    """Renumber cells: old cell i becomes newidx[i].

    Faces are re-oriented so that owner < neighbour (swapping upper and lower
    where the orientation flips) and re-sorted by (owner, neighbour).
    """
    newidx = np.asarray(newidx, dtype=np.int64)
    o = newidx[case.owner]
    nb = newidx[case.neighbour]
    flip = o > nb
    own2 = np.where(flip, nb, o)
    nb2 = np.where(flip, o, nb)
    up2 = np.where(flip, case.lower, case.upper)
    lo2 = np.where(flip, case.upper, case.lower)
    order = np.lexsort((nb2, own2))
    diag2 = np.empty_like(case.diag)
    diag2[newidx] = case.diag
    rhs2 = []
    for b in case.rhs:
        bb = np.empty_like(b)
        bb[newidx] = b
        rhs2.append(bb)
    meta = dict(case.meta)
    if "p_exact" in meta:
        pe = np.empty_like(meta["p_exact"])
        pe[newidx] = meta["p_exact"]
        meta["p_exact"] = pe
    meta["relabel"] = newidx
    return LduCase(name or case.name, case.n_cells,
                   own2[order].astype(np.int32), nb2[order].astype(np.int32),
                   diag2, up2[order].copy(), lo2[order].copy(), rhs2,
                   case.singular, meta)


def random_order(n: int, rng) -> np.ndarray:
    """A seeded random renumbering: cell i -> newidx[i]."""
    return rng.permutation(n).astype(np.int64)


def rcm_order(case: LduCase) -> np.ndarray:
    """Reverse Cuthill-McKee renumbering of the face graph (input ordering only).

    scipy's RCM returns perm with perm[k] = old cell placed at position k; the
    relabel map is its inverse.
    """
    import scipy.sparse as sp
    from scipy.sparse.csgraph import reverse_cuthill_mckee

    n = case.n_cells
    rows = np.concatenate([case.owner, case.neighbour])
    cols = np.concatenate([case.neighbour, case.owner])
    g = sp.csr_matrix((np.ones(rows.size, np.int8), (rows, cols)), shape=(n, n))
    perm = reverse_cuthill_mckee(g, symmetric_mode=True)
    newidx = np.empty(n, np.int64)
    newidx[perm] = np.arange(n)
    return newidx


def box_case(nx, ny=None, nz=None, *, coeff="uniform", sigma=0.5, scale=1.0,
             dirichlet_x0=None, neumann=False, nonsym=0.0, seed=0,
             rhs="normal", n_rhs=1, name=None) -> LduCase:
    """A small general-purpose box system for tests.

    coeff: "uniform" (a_f = scale) or "lognormal" (a_f = scale*exp(sigma*N(0,1))).
    dirichlet_x0: boundary coefficient a_b on cells with ix = 0 (None: none).
    nonsym: if > 0, lower_f = upper_f * exp(nonsym*N(0,1)) (a non-symmetric A
    for transpose tests; the diagonal is made strictly dominant).
    """
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    rng = np.random.default_rng(seed)
    own, nb, _ = box_faces(nx, ny, nz)
    n = nx * ny * nz
    f = own.size
    if coeff == "uniform":
        a = np.full(f, float(scale))
    elif coeff == "lognormal":
        a = scale * np.exp(sigma * rng.standard_normal(f))
    else:
        raise ValueError(coeff)
    up = a.copy()
    lo = a.copy()
    if nonsym > 0:
        lo = a * np.exp(nonsym * rng.standard_normal(f))
    ab = None
    if dirichlet_x0 is not None:
        ab = np.zeros(n)
        ab[np.arange(n) % nx == 0] = dirichlet_x0
    diag = assemble_diag(n, own, nb, up, lo, ab)
    if nonsym > 0:
        # strict dominance keeps the non-symmetric test matrices well posed
        colsum = np.bincount(own, weights=lo, minlength=n) + np.bincount(
            nb, weights=up, minlength=n)
        diag = -np.maximum(-diag, colsum) * 1.25
    rhss = []
    for _ in range(n_rhs):
        if rhs == "normal":
            rhss.append(rng.standard_normal(n))
        else:
            rhss.append(rng.uniform(-1.0, 1.0, n))
    singular = (dirichlet_x0 is None) and nonsym == 0
    case = LduCase(name or f"box{nx}x{ny}x{nz}", n, own, nb, diag, up, lo,
                   rhss, singular, {"shape": (nx, ny, nz)})
    if singular:
        case.rhs = [b - b.mean() for b in case.rhs]
    return case


# --------------------------------------------------------------------------
# The five benchmark workloads
# --------------------------------------------------------------------------

def _rng(c: int, s: int):
    return np.random.default_rng(1000 * c + s)


def _cell_centres(nx, ny, nz, h):
    i = np.arange(nx * ny * nz)
    ix = i % nx
    iy = (i // nx) % ny
    iz = i // (nx * ny)
    return (ix + 0.5) * h, (iy + 0.5) * h, (iz + 0.5) * h


def _csr_matvec(case: LduCase, x: np.ndarray) -> np.ndarray:
    """b = A x through scipy.sparse, used only to define manufactured rhs."""
    import scipy.sparse as sp

    n = case.n_cells
    rows = np.concatenate([np.arange(n), case.owner, case.neighbour])
    cols = np.concatenate([np.arange(n), case.neighbour, case.owner])
    vals = np.concatenate([case.diag, case.upper, case.lower])
    a = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    return a @ x


def config_c1(n=32) -> LduCase:
    """32^3 FD 7-point Laplacian, h = 1/n, a_f = 1/h^2; Dirichlet p = 0 at x = 0
    as a half-cell boundary coefficient 2/h^2; zero gradient elsewhere;
    b = A p_h with p = sin(pi x) cos(pi y) cos(pi z) sampled at cell centres,
    so the exact discrete solution is p_h."""
    h = 1.0 / n
    own, nb, _ = box_faces(n, n, n)
    N = n ** 3
    a = np.full(own.size, 1.0 / h ** 2)
    ab = np.zeros(N)
    ab[np.arange(N) % n == 0] = 2.0 / h ** 2
    diag = assemble_diag(N, own, nb, a, a, ab)
    x, y, z = _cell_centres(n, n, n, h)
    p = np.sin(np.pi * x) * np.cos(np.pi * y) * np.cos(np.pi * z)
    case = LduCase("c1", N, own, nb, diag, a.copy(), a.copy(), [], False,
                   {"shape": (n, n, n), "p_exact": p, "h": h})
    case.rhs = [_csr_matvec(case, p)]
    return case


def config_c2(n=128, order="random") -> LduCase:
    """128^3 pure zero-gradient box, a_f = exp(0.5 N(0,1)), cells renumbered by
    a seeded random permutation; order="rcm" adds an RCM renumbering on top.
    rhs ~ U[-1,1] minus its mean (a consistent singular system)."""
    own, nb, _ = box_faces(n, n, n)
    N = n ** 3
    a = np.exp(0.5 * _rng(2, 2).standard_normal(own.size))
    diag = assemble_diag(N, own, nb, a, a)
    case = LduCase("c2", N, own, nb, diag, a, a.copy(), [], True,
                   {"shape": (n, n, n)})
    case = relabel(case, random_order(N, _rng(2, 1)), "c2")
    b = _rng(2, 3).uniform(-1.0, 1.0, N)
    case.rhs = [b - b.mean()]
    if order == "rcm":
        case = relabel(case, rcm_order(case), "c2-rcm")
    return case


def c3_spacing(n=200):
    dx = 1.0 / n
    k = np.arange(n)
    dz = np.minimum((dx / 100.0) * 1.05 ** k, dx)
    return dx, dz


def config_c3(n=200, nxy=None) -> LduCase:
    """200^3 graded FV hex mesh: dx = dy = 1/n, dz_k = min((dx/100) 1.05^k, dx)
    (aspect ratio up to 100); FV coefficients a_x = a_y = dz_k,
    a_z = dx^2 / ((dz_k + dz_k+1)/2), times U[0.95, 1.05] per face; Dirichlet
    at the top layer with a_b = dx^2/(dz_top/2); zero gradient elsewhere;
    rhs ~ N(0,1)."""
    dx, dz = c3_spacing(n)
    m = n if nxy is None else nxy  # nxy < n: same z grading on a narrower box
    own, nb, ax = box_faces(m, m, n)
    N = m * m * n
    kz = own // (m * m)
    a = np.where(ax < 2, dz[kz],
                 dx * dx / (0.5 * (dz[kz] + dz[np.minimum(kz + 1, n - 1)])))
    a = a * _rng(3, 2).uniform(0.95, 1.05, own.size)
    ab = np.zeros(N)
    ab[np.arange(N) // (m * m) == n - 1] = dx * dx / (0.5 * dz[n - 1])
    diag = assemble_diag(N, own, nb, a, a, ab)
    b = _rng(3, 3).standard_normal(N)
    return LduCase("c3", N, own, nb, diag, a, a.copy(), [b], False,
                   {"shape": (m, m, n)})


def c3_assembly_inputs(n=200, nxy=None) -> dict:
    """Geometry and fields for assembling the c3 pressure equation on the GPU:
    the graded c3 box (dx = dy = 1/n, dz_k as c3), per internal face |S_f|,
    the delta coefficient 1/|d_f| and the owner's linear-interpolation weight
    w_f = (neighbour centre to face) / (centre to centre); per cell a
    diffusivity gamma = exp(0.3 N(0,1)) (seed s = 6, a stand-in for 1/A_p),
    the Dirichlet coefficient of the top layer gamma dx^2 / (dz_top / 2), a
    face flux phi ~ N(0,1) dx^2 (s = 7) and zero boundary fluxes."""
    dx, dz = c3_spacing(n)
    m = n if nxy is None else nxy
    own, nb, ax = box_faces(m, m, n)
    N = m * m * n
    kz = own // (m * m)
    kz1 = np.minimum(kz + 1, n - 1)
    mag_sf = np.where(ax < 2, dx * dz[kz], dx * dx)
    delta = np.where(ax < 2, 1.0 / dx, 1.0 / (0.5 * (dz[kz] + dz[kz1])))
    w = np.where(ax < 2, 0.5, dz[kz1] / (dz[kz] + dz[kz1]))
    gamma = np.exp(0.3 * _rng(3, 6).standard_normal(N))
    top = np.arange(N) // (m * m) == n - 1
    diag_bc = np.where(top, gamma * dx * dx / (0.5 * dz[n - 1]), 0.0)
    phi = _rng(3, 7).standard_normal(own.size) * dx * dx
    return {"n": N, "owner": own, "neighbour": nb, "gamma": gamma, "weights": w,
            "mag_sf": mag_sf, "delta": delta, "diag_bc": diag_bc, "phi": phi,
            "b_bc": np.zeros(N), "shape": (m, m, n)}


def config_c4(n=256, order="rcm") -> LduCase:
    """256^3 box, a_f = exp(N(0,1)), Dirichlet at x = 0 with a_b = 2, RCM
    numbering; three rhs ~ N(0,1) solved back to back with warm starts."""
    own, nb, _ = box_faces(n, n, n)
    N = n ** 3
    a = np.exp(_rng(4, 2).standard_normal(own.size))
    ab = np.zeros(N)
    ab[np.arange(N) % n == 0] = 2.0
    diag = assemble_diag(N, own, nb, a, a, ab)
    rhs = [np.random.default_rng(4000 + s).standard_normal(N) for s in (3, 13, 23)]
    case = LduCase("c4", N, own, nb, diag, a, a.copy(), rhs, False,
                   {"shape": (n, n, n)})
    if order == "rcm":
        case = relabel(case, rcm_order(case), "c4")
    return case


def config_c5(n=100) -> LduCase:
    """100^3 box, a_f = exp(0.5 N(0,1)), Dirichlet at x = 0 (a_b = 2); rhs and
    adjoint target x_t ~ N(0,1); 20 seeded faces for finite differences."""
    own, nb, _ = box_faces(n, n, n)
    N = n ** 3
    a = np.exp(0.5 * _rng(5, 2).standard_normal(own.size))
    ab = np.zeros(N)
    ab[np.arange(N) % n == 0] = 2.0
    diag = assemble_diag(N, own, nb, a, a, ab)
    b = _rng(5, 3).standard_normal(N)
    xt = _rng(5, 4).standard_normal(N)
    fd = np.sort(_rng(5, 5).choice(own.size, 20, replace=False))
    return LduCase("c5", N, own, nb, diag, a, a.copy(), [b], False,
                   {"shape": (n, n, n), "x_target": xt, "fd_faces": fd,
                    "a_boundary": ab})


def config_c5u(n=100, velocity=(1.0, 0.5, 0.25), courant=2.0) -> LduCase:
    """Non-symmetric stand-in for the velocity / turbulence systems the paper
    solves with PBiCG: one implicit Euler step of u_t + div(U u) =
    div(nu grad u) on the c5 box (h = 1/n), finite volumes with upwind
    convection.  Per face f (owner -> neighbour along axis k): diffusion
    D_f = nu_f h with nu_f = exp(0.5 N(0,1)) / n (seed s = 2, as c5), flux
    F_f = U_k h^2 >= 0; upper_f = -D_f, lower_f = -(D_f + F_f).  The diagonal
    holds each cell's outflow coefficients (D_f + F_f for the owner, D_f for
    the neighbour), h^3 / dt with dt = courant h / |U|, the upwind outflow
    U_k h^2 on the boundary faces at the far end of each axis, and a
    Dirichlet diffusion coefficient 2 mean(nu) h on the x = 0 inflow face.
    Column sums are non-negative: an M-matrix.  rhs N(0,1) (s = 3)."""
    own, nb, ax = box_faces(n, n, n)
    N = n ** 3
    h = 1.0 / n
    nu = np.exp(0.5 * _rng(5, 2).standard_normal(own.size)) / n
    U = np.asarray(velocity, dtype=np.float64)
    D = nu * h
    F = U[ax] * h * h
    up = -D
    lo = -(D + F)
    dt = courant * h / np.linalg.norm(U)
    diag = np.full(N, h ** 3 / dt)
    # outflow from the owner through f is D + F, from the neighbour D
    np.add.at(diag, own, D + F)
    np.add.at(diag, nb, D)
    i = np.arange(N)
    ijk = (i % n, (i // n) % n, i // (n * n))
    for k in range(3):
        diag[ijk[k] == n - 1] += U[k] * h * h
    diag[ijk[0] == 0] += 2.0 * nu.mean() * h
    b = _rng(5, 3).standard_normal(N)
    return LduCase("c5u", N, own, nb, diag, up, lo, [b], False,
                   {"shape": (n, n, n), "velocity": tuple(U), "courant": courant})


def config_case(name: str, **kw) -> LduCase:
    return {"c1": config_c1, "c2": config_c2, "c3": config_c3,
            "c4": config_c4, "c5": config_c5, "c5u": config_c5u}[name](**kw)
