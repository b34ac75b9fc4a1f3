"""CPU oracle of the geometry-embedding hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the GPU
library: the C sources here (exact.c, embed.c) are compiled on their own into
liboracle.so and evaluate the plain definitions with exact predicates.

What each function follows (section names of the paper):
  classify_blocks / solid_points  -- a cell is solid iff its centre lies in the
      closed solid bounded by the mesh ("Solid Voxelization Approaches":
      ray-cast parity; "Partial Surface Voxelization").  Points on the surface
      are solid; the +x ray is symbolically perturbed (simulation of
      simplicity) so parity never depends on rays grazing edges or vertices.
  refine -- "Refinement Flagging and Propagation": solid-boundary blocks,
      solid-adjacent blocks, N_prop propagation passes (Eq. 3), 2:1 eligibility.
  links -- "Boundary Cell Identification" and "Link-Length Computation": a
      fluid cell with a solid lattice neighbour has a cut link whose length q is
      the nearest surface crossing along the link, as a fraction of the link.
  grad -- derivative of q with respect to the hit triangle's vertices
      (closed form; not in the paper).
  links_dense -- "Memory Allocations for Boundary Cells": the per-block layout.
  bounce_back -- the linear interpolated bounce-back of Bouzidi et al. that
      the link lengths serve (Related Work), and simple bounce-back.
  solid_change -- cells whose solid flag a moving geometry changes
      (Limitations and Future Work: uncovered nodes become fluid).
  embed2d and the *2d functions -- the quadtree form the paper says the
      method covers (4x4 blocks, four children, D2Q9), on polygons given by
      edges (embed2d.c).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, f) for f in ("exact.c", "embed.c", "embed2d.c")]
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2 -fopenmp)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-Wno-unused-variable", "-Wno-maybe-uninitialized", *_SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i64, i32, dbl = C.c_int64, C.c_int, C.c_double
        L.or_orient2d.argtypes = [dbl] * 6
        L.or_orient2d_exact.argtypes = [dbl] * 6
        L.or_orient3d.argtypes = [P] * 4
        L.or_orient3d_exact.argtypes = [P] * 4
        L.or_orient3d_value.argtypes = [P] * 4
        L.or_orient3d_value.restype = dbl
        L.or_solid_points_brute.argtypes = [P, P, i32, i64, P, P]
        L.or_solid_points.argtypes = [P, P, i32, P, i64, P, P]
        L.or_classify_blocks.argtypes = [P, P, i32, P, i32, i64, P, i32, P]
        L.or_refine.argtypes = [P, i32, i64, P, P, i32, P, P, P, P]
        L.or_refine.restype = i64
        L.or_links.argtypes = [P, P, i32, P, i32, i64, P, i32, i64, P, P, P, P, P, P]
        L.or_links.restype = i64
        L.or_q_points.argtypes = [P, P, i32, P, i32, i64, P, P, P, P, P]
        L.or_grad.argtypes = [P, P, i32, P, i32, i64, P, i64, P, P, P, P, i32, P]
        L.or_q_given.argtypes = [P, P, i32, P, i32, i64, P, P, P, P, P]
        L.or_num_threads.restype = i32
        L.or_last_timing.argtypes = [P]
        L.or_set_threads.argtypes = [i32]
        L.or2_solid_point.argtypes = [P, P, P, i32, P]
        L.or2_classify_blocks.argtypes = [P, P, i32, P, i32, i64, P, i32, P]
        L.or2_refine.argtypes = [P, i32, i64, P, P, i32, P, P, P, P]
        L.or2_refine.restype = i64
        L.or2_links.argtypes = [P, P, i32, P, i32, i64, P, i64, P, P, P, P, P, P]
        L.or2_links.restype = i64
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _mesh_arrays(mesh):
    V = np.ascontiguousarray(mesh.verts, dtype=np.float64)  # float32 -> float64 is exact
    T = np.ascontiguousarray(mesh.tris, dtype=np.int32)
    return V, T


def orient2d(a, b, c) -> int:
    return lib().or_orient2d(float(a[0]), float(a[1]), float(b[0]), float(b[1]),
                             float(c[0]), float(c[1]))


def orient3d(a, b, c, d, exact_only: bool = False) -> int:
    arr = [np.ascontiguousarray(x, dtype=np.float64) for x in (a, b, c, d)]
    f = lib().or_orient3d_exact if exact_only else lib().or_orient3d
    return f(*[_p(x) for x in arr])


def num_threads() -> int:
    return lib().or_num_threads()


def set_threads(n: int) -> None:
    """OpenMP thread count of later oracle calls."""
    lib().or_set_threads(int(n))


def last_timing() -> dict:
    """Wall seconds of the last solid_points / q_points call: its bucket
    build, and the queries after it."""
    out = np.zeros(2, np.float64)
    lib().or_last_timing(_p(out))
    return {"build_s": float(out[0]), "query_s": float(out[1])}


# ----------------------------------------------------------------------------
# grid helpers
# ----------------------------------------------------------------------------

def level0_blocks(n0) -> np.ndarray:
    """All level-0 blocks, bx fastest."""
    nb = [n // 4 for n in n0]
    z, y, x = np.meshgrid(np.arange(nb[2]), np.arange(nb[1]), np.arange(nb[0]), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], 1).astype(np.int32)


def n_prop(d_spec: float) -> int:
    """Eq. 3 with the block length 4*dx_L: the 1/2^L factor cancels, leaving
    N_prop = 1 + floor(d_spec / (4 sqrt(2))) in base-cell units; the floor is
    taken exactly (largest k with 32 k^2 <= d_spec^2)."""
    d = Fraction(d_spec)
    if d <= 0:
        return 1
    k = int(float(d) / (4 * 2 ** 0.5))
    while 32 * (k + 1) ** 2 <= d * d:
        k += 1
    while k > 0 and 32 * k ** 2 > d * d:
        k -= 1
    return 1 + k


def cell_centres(bcoord: np.ndarray, L: int) -> np.ndarray:
    """[nb, 64, 3] cell centres, t = I + 4J + 16K."""
    t = np.arange(64)
    I = np.stack([t & 3, (t >> 2) & 3, t >> 4], 1)
    cells = 4 * bcoord[:, None, :].astype(np.int64) + I[None]
    return (cells + 0.5) * 2.0 ** (-L)


# ----------------------------------------------------------------------------
# classification
# ----------------------------------------------------------------------------

def solid_points(mesh, n0, pts: np.ndarray, brute: bool = False) -> np.ndarray:
    V, T = _mesh_arrays(mesh)
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(len(pts), dtype=np.uint8)
    n0a = np.ascontiguousarray(n0, dtype=np.int32)
    if brute:
        lib().or_solid_points_brute(_p(V), _p(T), T.shape[0], len(pts), _p(pts), _p(out))
    else:
        lib().or_solid_points(_p(V), _p(T), T.shape[0], _p(n0a), len(pts), _p(pts), _p(out))
    return out


def classify_blocks(mesh, n0, L: int, bcoord: np.ndarray, halo: bool = False) -> np.ndarray:
    V, T = _mesh_arrays(mesh)
    bc = np.ascontiguousarray(bcoord, dtype=np.int32)
    w = 216 if halo else 64
    out = np.zeros((len(bc), w), dtype=np.uint8)
    n0a = np.ascontiguousarray(n0, dtype=np.int32)
    lib().or_classify_blocks(_p(V), _p(T), T.shape[0], _p(n0a), L, len(bc), _p(bc),
                             1 if halo else 0, _p(out))
    return out


def pack_bits(solid_cells: np.ndarray) -> np.ndarray:
    """[nb, 64] uint8 -> [nb] uint64 with bit t = cell t."""
    w = (solid_cells.astype(np.uint64) & np.uint64(1)) << np.arange(64, dtype=np.uint64)
    return np.bitwise_or.reduce(w, axis=1)


# ----------------------------------------------------------------------------
# refinement
# ----------------------------------------------------------------------------

def refine(n0, L: int, bcoord: np.ndarray, solid_cells: np.ndarray, nprop: int) -> dict:
    bc = np.ascontiguousarray(bcoord, dtype=np.int32)
    nb = len(bc)
    s = np.ascontiguousarray(solid_cells, dtype=np.uint8)
    bclass = np.zeros(nb, np.uint8)
    ref = np.zeros(nb, np.uint8)
    cmap = np.zeros(nb, np.int32)
    child = np.zeros((8 * nb, 3), np.int32)
    n0a = np.ascontiguousarray(n0, dtype=np.int32)
    nch = lib().or_refine(_p(n0a), L, nb, _p(bc), _p(s), int(nprop), _p(bclass), _p(ref),
                          _p(cmap), _p(child))
    return {"bclass": bclass, "refine": ref, "child_map": cmap, "children": child[:nch].copy()}


# ----------------------------------------------------------------------------
# links
# ----------------------------------------------------------------------------

def links(mesh, n0, L: int, bcoord: np.ndarray, lattice: int) -> dict:
    V, T = _mesh_arrays(mesh)
    bc = np.ascontiguousarray(bcoord, dtype=np.int32)
    nb = len(bc)
    n0a = np.ascontiguousarray(n0, dtype=np.int32)
    mask = np.zeros(nb * 64, np.uint32)
    cap = 0
    args = lambda cap, arrs: [_p(V), _p(T), T.shape[0], _p(n0a), L, nb, _p(bc), lattice, cap,
                              _p(mask)] + [_p(a) for a in arrs]
    arrs = [np.zeros(1, np.int32), np.zeros(1, np.uint8), np.zeros(1, np.float64),
            np.zeros(1, np.int32), np.zeros(1, np.uint8)]
    n = lib().or_links(*args(0, arrs))
    arrs = [np.zeros(max(n, 1), np.int32), np.zeros(max(n, 1), np.uint8),
            np.zeros(max(n, 1), np.float64), np.zeros(max(n, 1), np.int32),
            np.zeros(max(n, 1), np.uint8)]
    n2 = lib().or_links(*args(n, arrs))
    assert n2 == n
    return {"mask": mask.reshape(nb, 64), "n": int(n), "cell": arrs[0][:n], "dir": arrs[1][:n],
            "q": arrs[2][:n], "tri": arrs[3][:n], "tied": arrs[4][:n]}


def q_points(mesh, n0, L: int, cells: np.ndarray, dirs: np.ndarray) -> dict:
    V, T = _mesh_arrays(mesh)
    cells = np.ascontiguousarray(cells, dtype=np.int32).reshape(-1, 3)
    dirs = np.ascontiguousarray(dirs, dtype=np.uint8)
    n = len(cells)
    q = np.zeros(n, np.float64)
    tri = np.zeros(n, np.int32)
    tied = np.zeros(n, np.uint8)
    n0a = np.ascontiguousarray(n0, dtype=np.int32)
    lib().or_q_points(_p(V), _p(T), T.shape[0], _p(n0a), L, n, _p(cells), _p(dirs), _p(q),
                      _p(tri), _p(tied))
    return {"q": q, "tri": tri, "tied": tied}


def q_given(mesh, n0, L: int, cells: np.ndarray, dirs: np.ndarray, tris: np.ndarray) -> dict:
    """For links given by cell index triples and directions, and a triangle
    named for each: the exact hit parameter of that triangle along the link
    (-1 if the closed segment misses it) and whether it equals the nearest
    hit exactly (the named triangle is one of the minimisers)."""
    V, T = _mesh_arrays(mesh)
    cells = np.ascontiguousarray(cells, dtype=np.int32).reshape(-1, 3)
    dirs = np.ascontiguousarray(dirs, dtype=np.uint8)
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    n = len(cells)
    q = np.zeros(n, np.float64)
    is_min = np.zeros(n, np.uint8)
    n0a = np.ascontiguousarray(n0, dtype=np.int32)
    lib().or_q_given(_p(V), _p(T), T.shape[0], _p(n0a), L, n, _p(cells), _p(dirs), _p(tris), _p(q), _p(is_min))
    return {"q": q, "is_min": is_min.astype(bool)}


def grad(mesh, n0, L: int, bcoord: np.ndarray, link_cell, link_dir, link_tri, w,
         absolute: bool = False) -> np.ndarray:
    """dL/dv for L = sum_i w_i q_i (closed form, see or_grad).  absolute=True
    sums |w_i| |dq_i/dv| instead: per component, the scale G_abs against which
    a float32 scatter-add of the same terms is judged."""
    V, T = _mesh_arrays(mesh)
    bc = np.ascontiguousarray(bcoord, dtype=np.int32)
    lc = np.ascontiguousarray(link_cell, dtype=np.int32)
    ld = np.ascontiguousarray(link_dir, dtype=np.uint8)
    lt = np.ascontiguousarray(link_tri, dtype=np.int32)
    ww = np.ascontiguousarray(w, dtype=np.float64)
    g = np.zeros((V.shape[0], 3), np.float64)
    n0a = np.ascontiguousarray(n0, dtype=np.int32)
    lib().or_grad(_p(V), _p(T), V.shape[0], _p(n0a), L, len(bc), _p(bc), len(lc), _p(lc), _p(ld),
                  _p(lt), _p(ww), 1 if absolute else 0, _p(g))
    return g


def lattice_dirs(lattice: int) -> np.ndarray:
    """Directions k = (cx+1) + 3(cy+1) + 9(cz+1) of D3Q19 (|c|^2 <= 2) or
    D3Q27, rest direction k = 13 left out, in increasing k."""
    ks = []
    for k in range(27):
        c = np.array([k % 3 - 1, (k // 3) % 3 - 1, k // 9 - 1])
        if k != 13 and (lattice == 27 or (c * c).sum() <= 2):
            ks.append(k)
    return np.array(ks)


def links_dense(nblocks: int, link_cell, link_dir, link_q, link_tri, lattice: int) -> dict:
    """Dense per-block layout of a link table (Methodology, "Memory
    Allocations for Boundary Cells"): boundary blocks are the blocks with at
    least one link, numbered in block order; block_map[b] is that number or
    -1.  q and tri are [nbnd, Q, 64] (direction s = position of the link's k
    among the lattice's directions, cell t), -1 where there is no link."""
    cell = np.asarray(link_cell, dtype=np.int64)
    blocks = np.unique(cell // 64)
    block_map = np.full(nblocks, -1, np.int32)
    block_map[blocks] = np.arange(len(blocks), dtype=np.int32)
    dirs = lattice_dirs(lattice)
    slot = np.full(27, -1, np.int64)
    slot[dirs] = np.arange(len(dirs))
    q = np.full((len(blocks), len(dirs), 64), -1.0, np.float32)
    tri = np.full((len(blocks), len(dirs), 64), -1, np.int32)
    j = block_map[cell // 64]
    s = slot[np.asarray(link_dir, dtype=np.int64)]
    q[j, s, cell % 64] = np.asarray(link_q, dtype=np.float32)
    tri[j, s, cell % 64] = np.asarray(link_tri, dtype=np.int32)
    return {"block_map": block_map, "q": q, "tri": tri}


def bounce_back(n0, L: int, bcoord, solid_cells, link_cell, link_dir, link_q, lattice: int, interpolate: bool,
                f_post, f_new):
    """Boundary step of a lattice Boltzmann solver at the links of a level
    (Related Work: linear interpolated bounce-back of Bouzidi et al., which
    needs the boundary node and one upstream fluid node per direction).

    For the link of fluid node x in direction p with length fraction q and
    the opposite direction pb (c_pb = -c_p), the population of x in direction
    pb after streaming is
      simple bounce-back:  f*_p(x)
      q <  1/2:  f*_p interpolated linearly at x - (1 - 2q) c_p between x and
                 the upstream node x - c_p:  2q f*_p(x) + (1 - 2q) f*_p(x - c_p)
      q >= 1/2:  the reflected f*_p(x), now at x + (2q - 1) c_p, and f*_pb(x),
                 at x - c_p after streaming, interpolated linearly at x:
                 f*_p(x) / (2q) + (1 - 1/(2q)) f*_pb(x)
    Where q < 1/2 and x - c_p is solid or in no block of the level, the one
    fluid node that form needs is not there and the link takes simple
    bounce-back (the q >= 1/2 form would extrapolate with a weight
    1 - 1/(2q) that is unbounded as q -> 0).

    Populations are [nblocks, Qf, 64] (directions in increasing k, rest
    included), arithmetic in float64 on the given values; the q < 1/2
    decision is taken on q as given (float32 in the table).  Returns
    (f_new as float64 with the link entries replaced, number of links that
    took the fallback)."""
    dirs = sorted(set(lattice_dirs(lattice).tolist()) | {13})
    slot = np.full(27, -1, np.int64)
    slot[dirs] = np.arange(len(dirs))
    out = np.array(f_new, dtype=np.float64, copy=True)
    fpost = np.asarray(f_post, dtype=np.float64)
    cell = np.asarray(link_cell, dtype=np.int64)
    k = np.asarray(link_dir, dtype=np.int64)
    qv = np.asarray(link_q)
    if len(cell) == 0:
        return out, 0
    b, t = cell // 64, cell % 64
    c = np.stack([k % 3 - 1, (k // 3) % 3 - 1, k // 9 - 1], axis=1)
    # the opposite direction, found from its vector
    cb = -c
    kb = (cb[:, 0] + 1) + 3 * (cb[:, 1] + 1) + 9 * (cb[:, 2] + 1)
    local = np.stack([t % 4, (t // 4) % 4, t // 16], axis=1)
    x = 4 * np.asarray(bcoord, dtype=np.int64)[b] + local
    fp = fpost[b, slot[k], t]
    fb = fpost[b, slot[kb], t]
    if not interpolate:
        out[b, slot[kb], t] = fp
        return out, 0
    # upstream node x - c_p: its block (if the level has it) and its cell
    u = x - c
    ubc = u // 4
    ncell = np.array([int(v) << L for v in n0], dtype=np.int64)
    inside = np.all((u >= 0) & (u < ncell[None, :]), axis=1)
    nbx = ncell // 4
    key = lambda a: (a[:, 2] * nbx[1] + a[:, 1]) * nbx[0] + a[:, 0]
    bkeys = key(np.asarray(bcoord, dtype=np.int64))
    order = np.argsort(bkeys)
    uk = key(ubc)
    pos = np.clip(np.searchsorted(bkeys[order], uk), 0, len(order) - 1)
    ub = order[pos]
    exists = inside & (bkeys[ub] == uk)
    ul = u - 4 * ubc
    ut = ul[:, 0] + 4 * ul[:, 1] + 16 * ul[:, 2]
    up_fluid = exists & (np.asarray(solid_cells)[ub, ut] == 0)
    fu = fpost[ub, slot[k], ut]
    q = qv.astype(np.float64)
    near = qv < 0.5
    use_up = near & up_fluid
    v = np.where(near, np.where(use_up, 2.0 * q * fp + (1.0 - 2.0 * q) * fu, fp),
                 fp / (2.0 * q) + (1.0 - 1.0 / (2.0 * q)) * fb)
    out[b, slot[kb], t] = v
    return out, int(np.count_nonzero(near & ~up_fluid))


def solid_change(mesh_prev, n0, L: int, bcoord, solid_cells) -> dict:
    """Cells of the blocks bcoord of level L whose solid flag differs between
    the previous mesh and the current classification solid_cells ([nb, 64],
    1 = solid): spawned = solid before and fluid now (nodes the geometry
    uncovered, which a solver must initialise), covered = fluid before and
    solid now.  The previous mesh is evaluated at the current cell centres by
    the same point rule as every solid flag.  Returns [nb, 64] uint8 masks and
    their counts."""
    before = classify_blocks(mesh_prev, n0, L, bcoord).astype(bool)
    now = np.asarray(solid_cells).astype(bool)
    spawned = before & ~now
    covered = now & ~before
    return {"spawned": spawned.astype(np.uint8), "covered": covered.astype(np.uint8),
            "n_spawned": int(spawned.sum()), "n_covered": int(covered.sum())}


# ----------------------------------------------------------------------------
# the whole path, level by level
# ----------------------------------------------------------------------------

def embed(mesh, n0, lf: int, lattice: int, d_spec: float = 2.0, with_links: bool = True) -> dict:
    """Level-by-level voxelization and refinement (levels 0..lf), then the
    cut-link table on level lf."""
    npr = n_prop(d_spec)
    bcoord = level0_blocks(n0)
    levels = []
    for L in range(lf + 1):
        cells = classify_blocks(mesh, n0, L, bcoord)
        rec = {"level": L, "bcoord": bcoord, "solid_cells": cells, "solid": pack_bits(cells)}
        if L < lf:
            r = refine(n0, L, bcoord, cells, npr)
            rec.update(r)
            bcoord = r["children"]
        levels.append(rec)
    out = {"levels": levels, "n_prop": npr}
    if with_links:
        out["links"] = links(mesh, n0, lf, levels[-1]["bcoord"], lattice)
    return out


# ----------------------------------------------------------------------------
# 2D: quadtrees of 4x4 blocks on polygons (vertices [nv, 2], edges [ne, 2])
# ----------------------------------------------------------------------------

def _poly_arrays(poly):
    V = np.ascontiguousarray(poly.verts, dtype=np.float64)
    E = np.ascontiguousarray(poly.edges, dtype=np.int32)
    return V, E


def level0_blocks2d(n0) -> np.ndarray:
    """All level-0 blocks of a 2D grid, bx fastest."""
    nbx, nby = n0[0] // 4, n0[1] // 4
    y, x = np.meshgrid(np.arange(nby), np.arange(nbx), indexing="ij")
    return np.stack([x.ravel(), y.ravel()], axis=1).astype(np.int32)


def solid_point2d(poly, p) -> int:
    """Point rule for one point, every edge a candidate."""
    V, E = _poly_arrays(poly)
    cand = np.arange(len(E), dtype=np.int32)
    pt = np.ascontiguousarray(p, dtype=np.float64)
    return int(lib().or2_solid_point(_p(V), _p(E), _p(cand), len(E), _p(pt)))


def classify_blocks2d(poly, n0, L: int, bcoord, halo: bool = False) -> np.ndarray:
    V, E = _poly_arrays(poly)
    bc = np.ascontiguousarray(bcoord, dtype=np.int32)
    w = 36 if halo else 16
    out = np.zeros((len(bc), w), dtype=np.uint8)
    n0a = np.ascontiguousarray(n0, dtype=np.int32)
    lib().or2_classify_blocks(_p(V), _p(E), len(E), _p(n0a), L, len(bc), _p(bc), 1 if halo else 0, _p(out))
    return out


def pack_bits16(solid_cells: np.ndarray) -> np.ndarray:
    """[nb, 16] -> [nb] uint16 with bit t = cell t."""
    w = (1 << np.arange(16, dtype=np.uint32)).astype(np.uint32)
    return (np.asarray(solid_cells, dtype=np.uint32) * w).sum(axis=1).astype(np.uint16)


def refine2d(n0, L: int, bcoord, solid_cells, nprop: int) -> dict:
    bc = np.ascontiguousarray(bcoord, dtype=np.int32)
    nb = len(bc)
    s = np.ascontiguousarray(solid_cells, dtype=np.uint8)
    bclass = np.zeros(nb, np.uint8)
    ref = np.zeros(nb, np.uint8)
    cmap = np.zeros(nb, np.int32)
    child = np.zeros((4 * nb, 2), np.int32)
    n0a = np.ascontiguousarray(n0, dtype=np.int32)
    nch = lib().or2_refine(_p(n0a), L, nb, _p(bc), _p(s), int(nprop), _p(bclass), _p(ref), _p(cmap), _p(child))
    return {"bclass": bclass, "refine": ref, "child_map": cmap, "children": child[:nch].copy()}


def links2d(poly, n0, L: int, bcoord) -> dict:
    V, E = _poly_arrays(poly)
    bc = np.ascontiguousarray(bcoord, dtype=np.int32)
    nb = len(bc)
    n0a = np.ascontiguousarray(n0, dtype=np.int32)
    mask = np.zeros(nb * 16, np.uint16)
    cap = 0
    n = lib().or2_links(_p(V), _p(E), len(E), _p(n0a), L, nb, _p(bc), cap, _p(mask), None, None, None, None, None)
    cell = np.zeros(max(n, 1), np.int32)
    dr = np.zeros(max(n, 1), np.uint8)
    q = np.zeros(max(n, 1), np.float64)
    edge = np.zeros(max(n, 1), np.int32)
    tied = np.zeros(max(n, 1), np.uint8)
    lib().or2_links(_p(V), _p(E), len(E), _p(n0a), L, nb, _p(bc), n, _p(mask), _p(cell), _p(dr), _p(q), _p(edge),
                    _p(tied))
    return {"n": int(n), "mask": mask, "cell": cell[:n], "dir": dr[:n], "q": q[:n], "tri": edge[:n],
            "tied": tied[:n]}


def embed2d(poly, n0, lf: int, d_spec: float = 2.0, with_links: bool = True) -> dict:
    """Level-by-level classification and refinement of a 2D grid (levels
    0..lf), then the D2Q9 cut-link table on level lf."""
    npr = n_prop(d_spec)
    bcoord = level0_blocks2d(n0)
    levels = []
    for L in range(lf + 1):
        cells = classify_blocks2d(poly, n0, L, bcoord)
        rec = {"level": L, "bcoord": bcoord, "solid_cells": cells, "solid": pack_bits16(cells)}
        if L < lf:
            r = refine2d(n0, L, bcoord, cells, npr)
            rec.update(r)
            bcoord = r["children"]
        levels.append(rec)
    out = {"levels": levels, "n_prop": npr}
    if with_links:
        out["links"] = links2d(poly, n0, lf, levels[-1]["bcoord"])
    return out
