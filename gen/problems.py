"""Seeded synthetic problem generator: grids, finite-volume Poisson matrices,
symmetry maps and right-hand sides.

This module produces *inputs only*.  It holds none of the solver's arithmetic
(no change of basis, no hierarchy, no Krylov iteration): it describes the
discrete problem that both the FP64 reference (``oracle/``) and the GPU
library receive.

Problem family (Sec. 2, model problem and stretching law; Sec. 5 random RHS):
cell-centred finite volumes with a two-point flux on a logically Cartesian
grid of the unit square/cube, homogeneous Dirichlet walls, optionally
tanh-stretched node coordinates, jittered nodes and a per-cell coefficient
kappa.  The grid carries ``s`` mirror symmetries about the mid-planes of the
first ``s`` axes (x, then y, then z).

Exact symmetry is built in, as the structure of Sec. 2 requires: every face
quantity is computed once on the *base mesh* (the 1/2^s fraction of the grid
with indices below N/2 along mirrored axes) and the full matrix is filled by
index mirroring, so mirrored entries are bit-identical.

Ordering conventions
--------------------
* base cell (i, j, k) has base index ``beta = i + Bx*(j + By*k)`` where
  ``B_t = N_t/2`` on mirrored axes and ``N_t`` otherwise;
* image ``a`` (0 <= a < 2^s) reflects axis t (``i -> N_t-1-i``) when bit t of
  ``a`` is set; image 0 is the base mesh;
* "mirrored" global ordering: row ``a*n_b + beta`` (the ordering of the
  paper's block structure, eqs. (2.2)-(2.5));
* "natural" global ordering: lexicographic ``i + Nx*(j + Ny*k)`` over the
  full grid.  ``img[beta, a]`` gives the global row of image a of base cell
  beta in whichever ordering the matrix is returned in.

Random fields are drawn in a fixed order (node jitter, kappa, RHS, target
field) from ``numpy.random.default_rng(seed)``; full-grid fields are drawn in
natural order and base-mesh fields in base order, so the draws do not depend
on the ordering the matrix is returned in.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np
import scipy.sparse as sp

# face kinds in BaseFaces.kind
FACE_INTERIOR = 0   # between two base cells
FACE_DIRICHLET = 1  # on the outer wall (homogeneous Dirichlet)
FACE_MIRROR = 2     # on a mirror plane, between a base cell and its reflection


@dataclasses.dataclass
class BaseFaces:
    """Geometry of every face touching a base-mesh cell.

    ``cell_a`` is always a base cell; ``cell_b`` is the other base cell for
    interior faces and -1 otherwise.  ``dist_a``/``dist_b`` are the distances
    from the cell centroids to the face centroid, ``area`` the face measure
    (an edge length in 2D).  ``axis`` is the normal axis; for mirror faces it
    is the mirrored axis, which is also the symmetry bit the face couples.
    """
    cell_a: np.ndarray
    cell_b: np.ndarray
    kind: np.ndarray
    axis: np.ndarray
    area: np.ndarray
    dist_a: np.ndarray
    dist_b: np.ndarray


@dataclasses.dataclass
class Problem:
    N: tuple                 # cells per axis, full grid
    s: int                   # number of mirror symmetries
    n: int                   # total unknowns
    n_b: int                 # base-mesh unknowns (n / 2^s)
    A: sp.csr_matrix         # full matrix in `ordering`
    img: np.ndarray          # (n_b, 2^s) int64, global row of image a of base cell
    b: np.ndarray            # (n, m) right-hand sides in `ordering`
    kappa_base: np.ndarray   # (n_b,) coefficient per base cell
    faces: BaseFaces
    ordering: str
    p_target: Optional[np.ndarray] = None   # (n,) target field for the adjoint loss
    nat_of_global: Optional[np.ndarray] = None  # natural index of each global row


def tanh_nodes(N: int, gamma: float) -> np.ndarray:
    """Node coordinates of the hyperbolic stretching law of Sec. 2 (eq. (2.26)),
    written 0-based: y_j = (1 + tanh(gamma (2j/N - 1)) / tanh(gamma)) / 2."""
    j = np.arange(N + 1, dtype=np.float64)
    return 0.5 * (1.0 + np.tanh(gamma * (2.0 * j / N - 1.0)) / np.tanh(gamma))


def _base_extents(N, s):
    D = len(N)
    B = []
    for t in range(D):
        if t < s:
            if N[t] % 2:
                raise ValueError("mirrored axes need an even cell count")
            B.append(N[t] // 2)
        else:
            B.append(N[t])
    return tuple(B)


def _node_coords(N, s, B, y_stretch, jitter, rng):
    """Node coordinates of the base region, shape (B_0+1, ..., B_{D-1}+1, D),
    indexed [i, j(, k), coord].  Jitter (if any) is drawn here, first."""
    D = len(N)
    axes = []
    for t in range(D):
        if t == 1 and y_stretch:
            c = tanh_nodes(N[t], y_stretch)
        else:
            c = np.arange(N[t] + 1, dtype=np.float64) / N[t]
        axes.append(c[: B[t] + 1])
    grids = np.meshgrid(*axes, indexing="ij")
    X = np.stack(grids, axis=-1)
    if jitter:
        shape = tuple(b + 1 for b in B)
        # one draw per base node and coordinate, in base-node lexicographic order
        # (i fastest), coordinate innermost
        nn = int(np.prod(shape))
        h = np.array([1.0 / N[t] for t in range(D)])
        J = rng.uniform(-jitter, jitter, size=(nn, D)) * h[None, :]
        J = J.reshape(tuple(reversed(shape)) + (D,))
        J = np.transpose(J, tuple(reversed(range(D))) + (D,))
        for t in range(D):
            # no normal motion on the outer walls or on mirror planes
            sl = [slice(None)] * D
            sl[t] = 0
            J[tuple(sl) + (t,)] = 0.0
            sl[t] = B[t]
            J[tuple(sl) + (t,)] = 0.0
        X = X + J
    return X


def _cell_index(idx, B):
    """Base index from per-axis base cell indices (i fastest)."""
    beta = np.zeros_like(idx[0])
    stride = 1
    for t in range(len(B)):
        beta = beta + idx[t] * stride
        stride *= B[t]
    return beta


def _base_geometry(N, s, B, X):
    """Cell centroids and every face of the base mesh."""
    D = len(N)
    # cell centroid = mean of the 2^D corner nodes
    sl0 = tuple(slice(0, B[t]) for t in range(D))
    cent = np.zeros(tuple(B) + (D,))
    for corner in range(1 << D):
        sl = tuple(slice((corner >> t) & 1, B[t] + ((corner >> t) & 1)) for t in range(D))
        cent += X[sl]
    cent /= float(1 << D)
    del sl0

    faces = {k: [] for k in ("a", "b", "kind", "axis", "area", "da", "db")}
    for e in range(D):
        # face planes normal to axis e at node index p = 0..B_e;
        # the face nodes span the other axes
        others = [t for t in range(D) if t != e]
        for p in range(B[e] + 1):
            # nodes of all faces on this plane: shape (B_o+1 ...) x D
            sl = [slice(None)] * D
            sl[e] = p
            Xp = X[tuple(sl)]  # shape: nodes over other axes, D
            if D == 2:
                o = others[0]
                n0 = Xp[:-1]
                n1 = Xp[1:]
                area = np.linalg.norm(n1 - n0, axis=-1)
                fc = 0.5 * (n0 + n1)
            else:
                o1, o2 = others
                p00 = Xp[:-1, :-1]
                p10 = Xp[1:, :-1]
                p11 = Xp[1:, 1:]
                p01 = Xp[:-1, 1:]
                d1 = p11 - p00
                d2 = p01 - p10
                area = 0.5 * np.linalg.norm(np.cross(d1, d2), axis=-1)
                fc = 0.25 * (p00 + p10 + p11 + p01)
            # the cells on either side of the plane
            face_shape = area.shape
            oidx = np.meshgrid(*[np.arange(B[t]) for t in others], indexing="ij")

            def full_idx(ce):
                idx = [None] * D
                for q, t in enumerate(others):
                    idx[t] = oidx[q]
                idx[e] = np.full(face_shape, ce, dtype=np.int64)
                return idx

            if p > 0:
                lo = full_idx(p - 1)
            if p < B[e]:
                hi = full_idx(p)

            def centroid(idx):
                return cent[tuple(idx)]

            if 0 < p < B[e]:
                ca, cb = lo, hi
                da = np.linalg.norm(fc - centroid(ca), axis=-1)
                db = np.linalg.norm(fc - centroid(cb), axis=-1)
                kind = FACE_INTERIOR
                a_idx, b_idx = _cell_index(ca, B), _cell_index(cb, B)
            elif p == 0:
                ca = hi
                da = np.linalg.norm(fc - centroid(ca), axis=-1)
                db = np.zeros_like(da)
                kind = FACE_DIRICHLET
                a_idx, b_idx = _cell_index(ca, B), np.full(face_shape, -1, dtype=np.int64)
            else:  # p == B[e]
                ca = lo
                da = np.linalg.norm(fc - centroid(ca), axis=-1)
                db = np.zeros_like(da)
                kind = FACE_MIRROR if e < s else FACE_DIRICHLET
                a_idx, b_idx = _cell_index(ca, B), np.full(face_shape, -1, dtype=np.int64)
            # store faces with the other-axis indices in Fortran (i fastest) order
            faces["a"].append(a_idx.ravel(order="F"))
            faces["b"].append(b_idx.ravel(order="F"))
            faces["kind"].append(np.full(area.size, kind, dtype=np.int8))
            faces["axis"].append(np.full(area.size, e, dtype=np.int8))
            faces["area"].append(area.ravel(order="F"))
            faces["da"].append(da.ravel(order="F"))
            faces["db"].append(db.ravel(order="F"))
    cat = {k: np.concatenate(v) for k, v in faces.items()}
    return BaseFaces(cat["a"].astype(np.int64), cat["b"].astype(np.int64), cat["kind"],
                     cat["axis"], cat["area"], cat["da"], cat["db"])


def transmissibility(faces: BaseFaces, kappa_base: np.ndarray) -> np.ndarray:
    """Two-point flux transmissibility of every base face.

    interior  T = |S| / (d_a/k_a + d_b/k_b)
    Dirichlet T = |S| k_a / d_a          (wall value at the face centroid)
    mirror    T = |S| k_a / (2 d_a)      (interior formula with the mirror
                                          image of the cell on the other side)
    """
    ka = kappa_base[faces.cell_a]
    T = np.empty(faces.area.shape)
    it = faces.kind == FACE_INTERIOR
    kb = kappa_base[faces.cell_b[it]]
    T[it] = faces.area[it] / (faces.dist_a[it] / ka[it] + faces.dist_b[it] / kb)
    dr = faces.kind == FACE_DIRICHLET
    T[dr] = faces.area[dr] * ka[dr] / faces.dist_a[dr]
    mi = faces.kind == FACE_MIRROR
    T[mi] = faces.area[mi] * ka[mi] / (2.0 * faces.dist_a[mi])
    return T


def base_blocks(faces: BaseFaces, T: np.ndarray, n_b: int, s: int):
    """The base-mesh blocks H_j (Sec. 2, eqs. (2.4)-(2.5) and the text after them):
    H_0 couples the base mesh with itself, H_{2^t} with its reflection about
    plane t (diagonal, one entry per cell touching that plane); all other H_j
    are zero for a two-point stencil.  Returns {j: csr}."""
    diag = np.zeros(n_b)
    # diagonal = sum of all face transmissibilities of the cell, accumulated
    # face-kind by face-kind in a fixed order (bitwise identical for every image)
    np.add.at(diag, faces.cell_a, T)
    it = faces.kind == FACE_INTERIOR
    np.add.at(diag, faces.cell_b[it], T[it])
    rows = np.concatenate([faces.cell_a[it], faces.cell_b[it], np.arange(n_b)])
    cols = np.concatenate([faces.cell_b[it], faces.cell_a[it], np.arange(n_b)])
    vals = np.concatenate([-T[it], -T[it], diag])
    H = {0: sp.csr_matrix((vals, (rows, cols)), shape=(n_b, n_b))}
    for t in range(s):
        mi = (faces.kind == FACE_MIRROR) & (faces.axis == t)
        H[1 << t] = sp.csr_matrix((-T[mi], (faces.cell_a[mi], faces.cell_a[mi])), shape=(n_b, n_b))
    for j in H:
        H[j].sort_indices()
    return H


def _natural_index(N, s, B, n_b):
    """nat[a, beta]: natural (lexicographic) index of image a of base cell beta."""
    D = len(N)
    grids = np.meshgrid(*[np.arange(B[t]) for t in range(D)], indexing="ij")
    base_idx = [g.ravel(order="F") for g in grids]  # beta order: i fastest
    nat = np.zeros((1 << s, n_b), dtype=np.int64)
    for a in range(1 << s):
        stride = 1
        tot = np.zeros(n_b, dtype=np.int64)
        for t in range(D):
            it = base_idx[t]
            if t < s and (a >> t) & 1:
                it = N[t] - 1 - it
            tot += it * stride
            stride *= N[t]
        nat[a] = tot
    return nat


def assemble_full(H: dict, n_b: int, s: int) -> sp.csr_matrix:
    """Full matrix in mirrored ordering from the base blocks: block (a, b) is
    H_{a xor b} (eqs. (2.4)-(2.5) generalised to 2^s subdomains)."""
    S = 1 << s
    out = None
    for j, Hj in H.items():
        if Hj.nnz == 0:
            continue
        a = np.arange(S)
        Pj = sp.csr_matrix((np.ones(S), (a, a ^ j)), shape=(S, S))
        term = sp.kron(Pj, Hj, format="csr")
        out = term if out is None else out + term
    out = out.tocsr()
    out.sort_indices()
    return out


def make_problem(N: Sequence[int], s: int, m: int = 1, seed: int = 0,
                 y_stretch: Optional[float] = None, jitter: Optional[float] = None,
                 kappa: str = "one", ordering: str = "natural",
                 with_target: bool = False, assemble: bool = True) -> Problem:
    """Build one seeded problem.

    N          cells per axis (2 or 3 axes)
    s          mirror symmetries (about the mid-planes of axes 0..s-1)
    m          right-hand sides, i.i.d. uniform[-1, 1] per cell (Sec. 5 uses a
               random RHS)
    y_stretch  gamma of the tanh law applied to the y nodes, or None
    jitter     node jitter amplitude in units of h (uniform[-j h, j h]) on the
               base mesh, mirrored; or None
    kappa      "one" or "lognormal" (lognormal(0,1) per base cell, mirrored)
    ordering   "natural" (lexicographic full grid) or "mirrored" (block order)
    assemble   False skips the full matrix (A = None): geometry, map and
               right-hand sides only
    """
    N = tuple(int(v) for v in N)
    D = len(N)
    if D not in (2, 3):
        raise ValueError("2D or 3D grids only")
    if not 0 <= s <= D:
        raise ValueError("s must be between 0 and the dimension")
    rng = np.random.default_rng(seed)
    B = _base_extents(N, s)
    n_b = int(np.prod(B))
    S = 1 << s
    n = n_b * S
    X = _node_coords(N, s, B, y_stretch, jitter, rng)
    faces = _base_geometry(N, s, B, X)
    if kappa == "one":
        kb = np.ones(n_b)
    elif kappa == "lognormal":
        kb = rng.lognormal(0.0, 1.0, size=n_b)
    else:
        raise ValueError(kappa)
    if assemble:
        T = transmissibility(faces, kb)
        H = base_blocks(faces, T, n_b, s)
        A_mir = assemble_full(H, n_b, s)
    nat = _natural_index(N, s, B, n_b)          # (S, n_b)
    nat_of_mir = nat.reshape(-1)                # mirrored row -> natural index
    b_nat = rng.uniform(-1.0, 1.0, size=(m, n)).T.copy()   # natural order, column by column
    p_nat = rng.standard_normal(n) if with_target else None
    if ordering == "mirrored":
        A = A_mir if assemble else None
        img = (np.arange(S)[None, :] * n_b + np.arange(n_b)[:, None]).astype(np.int64)
        b = b_nat[nat_of_mir]
        p_t = p_nat[nat_of_mir] if p_nat is not None else None
        nat_of_global = nat_of_mir
    elif ordering == "natural":
        A = None
        if assemble:
            perm = sp.csr_matrix((np.ones(n), (nat_of_mir, np.arange(n))), shape=(n, n))
            A = (perm @ A_mir @ perm.T).tocsr()
            A.sort_indices()
        img = nat.T.copy().astype(np.int64)
        b = b_nat
        p_t = p_nat
        nat_of_global = np.arange(n)
    else:
        raise ValueError(ordering)
    return Problem(N=N, s=s, n=n, n_b=n_b, A=A, img=np.ascontiguousarray(img), b=np.ascontiguousarray(b),
                   kappa_base=kb, faces=faces, ordering=ordering, p_target=p_t,
                   nat_of_global=nat_of_global)


# ---------------------------------------------------------------------------
# The workload family: five named configurations.  Seeds follow 240705930 + i.
# ---------------------------------------------------------------------------
CONFIG_SEED0 = 240705930


def config_problem(name: str, scale: Optional[int] = None, ordering: str = "natural",
                   assemble: bool = True) -> Problem:
    """Named workloads.  ``scale`` overrides the cell count per axis (for
    small parity instances of the same recipe)."""
    if name == "poisson2d_128_s1":
        N = scale or 128
        return make_problem((N, N), s=1, m=1, seed=CONFIG_SEED0 + 0, ordering=ordering)
    if name == "channel3d_128_s3":
        N = scale or 128
        return make_problem((N, N, N), s=3, m=4, seed=CONFIG_SEED0 + 1, y_stretch=1.5,
                            ordering=ordering)
    if name == "jitter3d_192_s3":
        N = scale or 192
        return make_problem((N, N, N), s=3, m=1, seed=CONFIG_SEED0 + 2, jitter=0.2,
                            kappa="lognormal", ordering=ordering, assemble=assemble)
    if name == "adjoint3d_256_s3":
        N = scale or 256
        return make_problem((N, N, N), s=3, m=1, seed=CONFIG_SEED0 + 4, kappa="lognormal",
                            ordering=ordering, with_target=True, assemble=assemble)
    raise KeyError(name)


def batch_problems(count: int = 64, seed: int = CONFIG_SEED0 + 3, n_min: int = 32, n_max: int = 96,
                   ordering: str = "natural"):
    """The batched workload: ``count`` cubic Dirichlet problems with N uniform
    over the even integers in [n_min, n_max], s uniform in {1,2,3} and m
    uniform in {1..8}; each system gets its own sub-seed."""
    rng = np.random.default_rng(seed)
    evens = np.arange(n_min, n_max + 1, 2)
    Ns = rng.choice(evens, size=count)
    ss = rng.integers(1, 4, size=count)
    ms = rng.integers(1, 9, size=count)
    subseeds = rng.integers(0, 2**31 - 1, size=count)
    out = []
    for i in range(count):
        N = int(Ns[i])
        out.append(make_problem((N, N, N), s=int(ss[i]), m=int(ms[i]), seed=int(subseeds[i]),
                                ordering=ordering))
    return out


# ---------------------------------------------------------------------------
# Repeated geometries: a domain made of copies of one subdomain
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class CopiesProblem:
    N: tuple                 # cells per axis of one copy
    copies: int              # number of copies placed side by side along axis 0
    n: int                   # total unknowns
    n_b: int                 # unknowns of one copy
    A: sp.csr_matrix         # full matrix, natural (lexicographic) order of the whole grid
    sub: np.ndarray          # (n_b, copies) int64: global row of cell i of the base copy in copy a
    b: np.ndarray            # (n, m) right-hand sides


def make_repeated_problem(N: Sequence[int], copies: int, m: int = 1, seed: int = 0, mirror: bool = False,
                          walls: str = "dirichlet", kappa: str = "lognormal") -> CopiesProblem:
    """``copies`` copies of an N grid of unit cells placed side by side along
    axis 0 (a repeated geometry; with ``mirror`` every odd copy is the mirror
    image of the base copy, a reflected geometry).  The coefficient of a cell
    (lognormal(0, 1) per cell of the base copy, or 1) is the same in every
    copy.  Cell-centred two-point fluxes with the harmonic mean of the two
    cells; homogeneous Dirichlet walls (flux 2 kappa h^(D-2)).  walls =
    "mixed" makes the boundary conditions differ between copies: the low wall
    of axis 1 is insulating (no flux) in every odd copy, and so is the wall
    closing the domain at the far end of axis 0.  Right-hand sides i.i.d.
    uniform[-1, 1] in natural order.  The diagonal sums opposite faces first,
    so a cell and its image carry the same bits."""
    N = tuple(int(v) for v in N)
    D = len(N)
    if D not in (2, 3) or copies < 1:
        raise ValueError("2D or 3D copies, at least one")
    rng = np.random.default_rng(seed)
    n_b = int(np.prod(N))
    full = (N[0] * copies,) + N[1:]
    n = n_b * copies
    kb = rng.lognormal(0.0, 1.0, size=n_b) if kappa == "lognormal" else np.ones(n_b)

    strides_full = np.cumprod((1,) + full[:-1])     # axis 0 fastest
    strides_base = np.cumprod((1,) + N[:-1])
    g_all = np.arange(n, dtype=np.int64)
    grid = np.stack([(g_all // strides_full[ax]) % full[ax] for ax in range(D)], axis=1)   # natural order
    copy_of = grid[:, 0] // N[0]
    x0 = grid[:, 0] % N[0]
    if mirror:
        x0 = np.where(copy_of % 2 == 1, N[0] - 1 - x0, x0)
    base_idx = x0 * strides_base[0]
    for ax in range(1, D):
        base_idx = base_idx + grid[:, ax] * strides_base[ax]
    kap = kb[base_idx]
    rows, cols, vals = [], [], []
    face = np.zeros((n, 2 * D))
    for ax in range(D):
        for side, step in ((0, -1), (1, 1)):
            f = 2 * ax + side
            nbc = grid[:, ax] + step
            inside = (nbc >= 0) & (nbc < full[ax])
            h = g_all + step * strides_full[ax]
            gi, hi = g_all[inside], h[inside]
            t = 1.0 / (0.5 / kap[gi] + 0.5 / kap[hi])
            face[gi, f] = t
            rows.append(gi)
            cols.append(hi)
            vals.append(-t)
            out = ~inside
            wall = 2.0 * kap[out]
            if walls == "mixed":
                if ax == 1 and side == 0:
                    wall = np.where(copy_of[out] % 2 == 1, 0.0, wall)
                if ax == 0 and side == 1:
                    wall = np.zeros_like(wall)
            face[out, f] = wall
    pairs = [face[:, 2 * ax] + face[:, 2 * ax + 1] for ax in range(D)]
    diag = pairs[0] + pairs[1]
    if D == 3:
        diag = diag + pairs[2]
    rows.append(g_all)
    cols.append(g_all)
    vals.append(diag)
    rows, cols, vals = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    A.sort_indices()
    sub = np.empty((n_b, copies), dtype=np.int64)
    sub[base_idx, copy_of] = np.arange(n)
    b = rng.uniform(-1.0, 1.0, size=(m, n)).T.copy()
    return CopiesProblem(N=N, copies=copies, n=n, n_b=n_b, A=A, sub=sub, b=np.ascontiguousarray(b))
