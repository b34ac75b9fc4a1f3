"""Cut-link sets derived from per-cell solid flags (test helper).

A fluid cell x of level L has a link in direction k iff the same-level
centre x + c_k is solid (Methodology, "Boundary Cell Identification").  Given
the oracle's solid flag of every cell of the level's blocks, the link mask of
a block follows from its 6^3 halo: halo centres inside existing blocks take
those blocks' flags, centres in the domain but in no block of the level are
classified by the oracle's point rule, centres outside the domain are fluid.
This gives the whole link set of a level (which links exist, in the table's
(block, t, k) order) without computing any q, so the GPU's set can be checked
for completeness at full size.

Only numpy and the oracle are used; nothing here comes from the GPU path.
"""
from __future__ import annotations

import numpy as np

import oracle

_OFF = np.array([[dx, dy, dz] for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)])


def _dirs(lattice: int) -> np.ndarray:
    return oracle.lattice_dirs(lattice)


class BlockIndex:
    """Lookup of level-L blocks by their coordinates: a dense index map over
    the blocks' bounding box (grown by one block), or sorted linear keys when
    that box is too large."""

    DENSE_MAX = 400_000_000

    def __init__(self, n0, L: int, bcoord: np.ndarray):
        self.dims = (np.asarray(n0, dtype=np.int64) // 4) << L
        self.bc = np.asarray(bcoord, dtype=np.int64)
        self.dense = None
        if len(self.bc):
            self.lo = self.bc.min(0) - 1
            self.ext = self.bc.max(0) + 2 - self.lo
            if int(np.prod(self.ext)) <= self.DENSE_MAX:
                self.dense = np.full(int(np.prod(self.ext)), -1, np.int32)
                self.dense[self._dkey(self.bc)] = np.arange(len(self.bc), dtype=np.int32)
        if self.dense is None:
            k = self.key(self.bc)
            self.order = np.argsort(k, kind="stable")
            self.skeys = k[self.order]

    def key(self, c: np.ndarray) -> np.ndarray:
        return (c[:, 2] * self.dims[1] + c[:, 1]) * self.dims[0] + c[:, 0]

    def _dkey(self, c: np.ndarray) -> np.ndarray:
        r = c - self.lo
        return (r[:, 2] * self.ext[1] + r[:, 1]) * self.ext[0] + r[:, 0]

    def find(self, c: np.ndarray):
        """(index or -1, in_domain) of the blocks at coordinates c."""
        c = np.asarray(c, dtype=np.int64)
        inside = ((c >= 0) & (c < self.dims[None, :])).all(1)
        idx = np.full(len(c), -1, np.int64)
        if not len(self.bc) or not inside.any():
            return idx, inside
        if self.dense is not None:
            r = c - self.lo
            inbox = inside & ((r >= 0) & (r < self.ext[None, :])).all(1)
            idx[inbox] = self.dense[self._dkey(c[inbox])]
            return idx, inside
        kq = self.key(c[inside])
        pos = np.clip(np.searchsorted(self.skeys, kq), 0, len(self.skeys) - 1)
        idx[inside] = np.where(self.skeys[pos] == kq, self.order[pos], -1)
        return idx, inside


def candidate_blocks(index: BlockIndex, solid_words: np.ndarray) -> np.ndarray:
    """Blocks that can hold a link: a fluid cell, and either a solid cell of
    their own or a 26-neighbour that is missing (in the domain, in no block of
    the level) or holds a solid cell.  Every other block is all solid (no
    fluid cell) or all fluid with all-fluid neighbours, so none of its halo
    centres is solid and it has no link."""
    w = np.asarray(solid_words).view(np.uint64)
    full = np.uint64(0xFFFFFFFFFFFFFFFF)
    has_fluid = w != full
    has_solid = w != 0
    near = has_solid.copy()
    for d in _OFF:
        if not d.any():
            continue
        idx, inside = index.find(index.bc + d)
        near |= inside & ((idx < 0) | has_solid[np.maximum(idx, 0)])
    return np.nonzero(has_fluid & near)[0]


def halo_flags(mesh, n0, L: int, index: BlockIndex, solid_words: np.ndarray, blocks: np.ndarray) -> np.ndarray:
    """[len(blocks), 6, 6, 6] solid flags (z, y, x) of the halo centres
    4 b + (-1..4) of the given blocks."""
    w = np.asarray(solid_words).view(np.uint64)
    nbk = len(blocks)
    H = np.zeros((nbk, 6, 6, 6), np.uint8)
    tb = np.arange(64, dtype=np.uint64)
    # halo index range fed by a neighbour offset d along one axis, and the
    # neighbour's local cells that feed it
    dst = {-1: slice(0, 1), 0: slice(1, 5), 1: slice(5, 6)}
    src = {-1: slice(3, 4), 0: slice(0, 4), 1: slice(0, 1)}
    pending_pts, pending_where = [], []
    for d in _OFF:
        idx, inside = index.find(index.bc[blocks] + d)
        sx, sy, sz = (dst[int(v)] for v in d)
        have = idx >= 0
        if have.any():
            bits = (w[idx[have]][:, None] >> tb[None, :]) & np.uint64(1)
            cells = bits.astype(np.uint8).reshape(-1, 4, 4, 4)   # [K][J][I]
            H[np.nonzero(have)[0][:, None, None, None],
              np.arange(6)[sz][None, :, None, None],
              np.arange(6)[sy][None, None, :, None],
              np.arange(6)[sx][None, None, None, :]] = cells[:, src[int(d[2])], src[int(d[1])], src[int(d[0])]]
        miss = np.nonzero(inside & ~have)[0]
        if len(miss):
            zz, yy, xx = np.meshgrid(np.arange(6)[sz], np.arange(6)[sy], np.arange(6)[sx], indexing="ij")
            loc = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1) - 1          # -1..4 in the block frame
            cc = 4 * index.bc[blocks[miss]][:, None, :] + loc[None, :, :]
            pending_pts.append(((cc + 0.5) * 2.0 ** -L).reshape(-1, 3))
            pending_where.append((miss, zz.ravel(), yy.ravel(), xx.ravel()))
    if pending_pts:
        flags = oracle.solid_points(mesh, n0, np.concatenate(pending_pts))
        o = 0
        for (miss, zz, yy, xx) in pending_where:
            n = len(miss) * len(zz)
            f = flags[o:o + n].reshape(len(miss), len(zz))
            o += n
            H[miss[:, None], zz[None, :], yy[None, :], xx[None, :]] = f
    return H


def link_masks(H: np.ndarray, lattice: int) -> np.ndarray:
    """[n, 64] uint32 link masks (bit k) of the blocks whose halos are H."""
    n = H.shape[0]
    centre = H[:, 1:5, 1:5, 1:5]
    m = np.zeros((n, 4, 4, 4), np.uint32)
    for k in _dirs(lattice):
        cx, cy, cz = k % 3 - 1, (k // 3) % 3 - 1, k // 9 - 1
        nb = H[:, 1 + cz:5 + cz, 1 + cy:5 + cy, 1 + cx:5 + cx]
        m |= ((nb != 0) & (centre == 0)).astype(np.uint32) << np.uint32(k)
    return m.reshape(n, 64)


def links_from_masks(blocks: np.ndarray, masks: np.ndarray):
    """(cell = block * 64 + t, dir) of every set bit, in (block, t, k) order."""
    flat = masks.reshape(-1)
    rows = []
    for k in range(27):
        pos = np.nonzero(flat & np.uint32(1 << k))[0]
        if len(pos):
            rows.append(pos.astype(np.int64) * 27 + k)
    if not rows:
        return np.zeros(0, np.int64), np.zeros(0, np.uint8)
    key = np.sort(np.concatenate(rows))
    pos, k = key // 27, key % 27
    cell = np.asarray(blocks, dtype=np.int64)[pos // 64] * 64 + pos % 64
    return cell, k.astype(np.uint8)


def level_link_set(mesh, n0, L: int, bcoord: np.ndarray, solid_words: np.ndarray, lattice: int):
    """The whole link set of a level: (cell, dir) in table order, the
    candidate blocks and their masks."""
    index = BlockIndex(n0, L, bcoord)
    cand = candidate_blocks(index, solid_words)
    masks = np.zeros((0, 64), np.uint32)
    cells, dirs = np.zeros(0, np.int64), np.zeros(0, np.uint8)
    chunk = 400000
    parts_c, parts_d, parts_m = [], [], []
    for s in range(0, len(cand), chunk):
        b = cand[s:s + chunk]
        m = link_masks(halo_flags(mesh, n0, L, index, solid_words, b), lattice)
        c, d = links_from_masks(b, m)
        parts_c.append(c)
        parts_d.append(d)
        parts_m.append(m)
    if parts_c:
        cells, dirs, masks = np.concatenate(parts_c), np.concatenate(parts_d), np.concatenate(parts_m)
    return {"cell": cells, "dir": dirs, "blocks": cand, "masks": masks}
