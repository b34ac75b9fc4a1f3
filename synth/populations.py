"""Seeded lattice populations and link tables for the bounce-back step.

Populations are laid out [nblocks][Qf][64]: cell t of block b in the s-th
direction of the lattice, directions k = (cx+1) + 3(cy+1) + 9(cz+1) in
increasing k with the rest direction (k = 13) included; Qf = 19 for D3Q19
(|c|^2 <= 2), 27 for D3Q27.  Values are lattice weights times (1 + noise),
the size of post-collision populations near rest.
"""
from __future__ import annotations

import numpy as np


def pop_dirs(lattice: int) -> np.ndarray:
    """Directions k of the population layout, increasing, rest included."""
    ks = np.arange(27)
    c = np.stack([ks % 3 - 1, (ks // 3) % 3 - 1, ks // 9 - 1], axis=1)
    n2 = (c * c).sum(1)
    return ks[n2 <= 2] if lattice == 19 else ks


def lattice_weights(lattice: int) -> np.ndarray:
    """Weights of the standard D3Q19 / D3Q27 lattices by |c|^2, in the
    population layout's direction order."""
    ks = pop_dirs(lattice)
    c = np.stack([ks % 3 - 1, (ks // 3) % 3 - 1, ks // 9 - 1], axis=1)
    n2 = (c * c).sum(1)
    table = {19: [1 / 3, 1 / 18, 1 / 36], 27: [8 / 27, 2 / 27, 1 / 54, 1 / 216]}[lattice]
    return np.array([table[v] for v in n2])


def populations(nblocks: int, lattice: int, seed: int, noise: float = 0.1, dtype=np.float32) -> np.ndarray:
    """[nblocks, Qf, 64] populations w_k (1 + noise * u), u uniform in [-1, 1)."""
    rng = np.random.default_rng(seed)
    w = lattice_weights(lattice)
    u = rng.uniform(-1.0, 1.0, size=(nblocks, len(w), 64))
    return (w[None, :, None] * (1.0 + noise * u)).astype(dtype)


def random_links(nblocks: int, lattice: int, seed: int, per_block: int = 40) -> dict:
    """A table of up to per_block links in each of the first blocks: distinct
    (cell, direction) pairs, q float32 in (0, 1] with the special values 1/2
    and 1 and some q close to 0, 1/2 and 1; sorted by (block, cell, direction)
    as the cut-link table is.  Not a geometry: any cell may hold a link."""
    rng = np.random.default_rng(seed)
    ks = pop_dirs(lattice)
    ks = ks[ks != 13]
    nb = min(nblocks, max(1, nblocks // 2))
    blocks = np.sort(rng.choice(nblocks, size=nb, replace=False))
    cells, dirs = [], []
    for b in blocks:
        pick = rng.choice(64 * len(ks), size=per_block, replace=False)
        cells.append(b * 64 + pick // len(ks))
        dirs.append(ks[pick % len(ks)])
    cell = np.concatenate(cells).astype(np.int64)
    dr = np.concatenate(dirs).astype(np.int64)
    order = np.lexsort((dr, cell))
    cell, dr = cell[order], dr[order]
    n = len(cell)
    q = rng.uniform(0.0, 1.0, n)
    special = rng.integers(0, 8, n)
    q = np.where(special == 0, 0.5, q)
    q = np.where(special == 1, 1.0, q)
    q = np.where(special == 2, 0.5 - rng.uniform(0, 1e-6, n), q)
    q = np.where(special == 3, 1e-6 * rng.uniform(0.5, 1.0, n), q)
    q = q.astype(np.float32)
    q = np.where(q <= 0, np.float32(1e-7), q).astype(np.float32)
    return {"cell": cell.astype(np.int32), "dir": dr.astype(np.uint8), "q": q}
