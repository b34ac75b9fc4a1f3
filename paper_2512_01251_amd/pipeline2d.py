"""Level-by-level driver of the 2D path (quadtrees of 4x4 blocks, polygons,
D2Q9) on top of the geo2_* entry points: for L = 0 .. L_f the ROWS bins and
the voxelization of level L, the refinement flags and children for L < L_f,
then on L_f the LINKS bins and the cut-link table.  As in 3D, the host waits
for the child count of each level and reads every bin and link count once at
the end; a pass that overflowed a buffer is redone with larger buffers."""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import (GEO_BINS_LINKS, GEO_BINS_ROWS, GEO_CALL2_BINS, GEO_CALL2_CUTLINKS, GEO_CALL2_REFINE,
               geo2_build_bins, geo2_cutlinks, geo2_level0_blocks, geo2_refine_flags, geo2_voxelize, geo_nprop,
               geo_workspace_size, make_bins, make_level2, make_mesh2)


@dataclass
class Level2D:
    level: int
    bcoord: torch.Tensor                 # int32 [nb, 2]
    rows_off: torch.Tensor = None
    rows_val: torch.Tensor = None
    solid: torch.Tensor = None           # int16 [nb] (bit t = cell t)
    bclass: torch.Tensor = None
    refine: torch.Tensor = None
    child_map: torch.Tensor = None


@dataclass
class Links2D:
    cell: torch.Tensor                   # int32 [n] (16 b + t)
    dir: torch.Tensor                    # uint8 [n] (D2Q9 k)
    q: torch.Tensor                      # float32 [n]
    edge: torch.Tensor                   # int32 [n]

    @property
    def n(self) -> int:
        return int(self.cell.shape[0])


@dataclass
class Embedding2D:
    n0: tuple
    lf: int
    levels: list = field(default_factory=list)
    links: Links2D = None


class Embedder2D:
    """Holds the workspace and remembered capacities across calls."""

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        self.ws = torch.empty(0, dtype=torch.uint8, device=self.device)
        self.caps: dict = {}
        self._host_n = torch.zeros(1, dtype=torch.int64, pin_memory=self.device.type == "cuda")

    def _workspace(self, nbytes: int) -> torch.Tensor:
        if self.ws.numel() < nbytes:
            self.ws = torch.empty(int(nbytes * 1.25) + 4096, dtype=torch.uint8, device=self.device)
        return self.ws

    def embed(self, verts: torch.Tensor, edges: torch.Tensor, n0, lf: int, d_spec: float = 2.0,
              with_links: bool = True) -> Embedding2D:
        for _ in range(lf + 4):
            out = self._embed_once(verts, edges, n0, lf, d_spec, with_links)
            if out is not None:
                return out
        raise RuntimeError("buffer capacities did not converge")

    def _bins(self, mesh, lvd, kind, nkeys, cap, d_count):
        dev = self.device
        off = torch.empty(nkeys + 1, dtype=torch.int32, device=dev)
        val = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        bins = make_bins(kind, nkeys, off, val, cap, d_count)
        geo2_build_bins(mesh, lvd, kind, bins, self._workspace(geo_workspace_size(GEO_CALL2_BINS, nkeys, 0)))
        return bins, off, val

    def _embed_once(self, verts, edges, n0, lf, d_spec, with_links):
        dev = self.device
        mesh = make_mesh2(verts, edges)
        n_prop = geo_nprop(d_spec)
        ctr = torch.zeros(2 * lf + 4, dtype=torch.int64, device=dev)
        cnt = lambda i: ctr[i:i + 1]
        checks = []
        bcoord = torch.empty(((n0[0] // 4) * (n0[1] // 4), 2), dtype=torch.int32, device=dev)
        geo2_level0_blocks(n0, bcoord)
        out = Embedding2D(tuple(n0), lf)
        child_maps = []
        rows = None

        def row_bins(L, lvd):
            # ROWS bins depend on the level, not on its blocks: the next level's
            # are enqueued before the host waits for that level's block count
            nkeys = n0[1] << L
            key = ("rows", L)
            cap = self.caps.get(key, max(1024, 4 * edges.shape[0]))
            bins, off, val = self._bins(mesh, lvd, GEO_BINS_ROWS, nkeys, cap, cnt(L))
            return key, cap, bins, off, val

        ahead = row_bins(0, make_level2(n0, 0, bcoord, child_maps))
        for L in range(lf + 1):
            lvd = make_level2(n0, L, bcoord, child_maps)
            rec = Level2D(L, bcoord)
            key, cap, rows, rec.rows_off, val = ahead
            rec.rows_val = val
            checks.append((L, cap, key, lambda c, rec=rec, val=val: setattr(rec, "rows_val", val[:c])))
            rec.solid = torch.empty(lvd.nblocks, dtype=torch.int16, device=dev)
            geo2_voxelize(mesh, lvd, rows, rec.solid)
            if L < lf:
                nb = lvd.nblocks
                rec.bclass = torch.empty(nb, dtype=torch.uint8, device=dev)
                rec.refine = torch.empty(nb, dtype=torch.uint8, device=dev)
                rec.child_map = torch.empty(nb, dtype=torch.int32, device=dev)
                child = torch.empty((4 * nb, 2), dtype=torch.int32, device=dev)
                d_n = cnt(lf + 1 + L)
                ws = self._workspace(geo_workspace_size(GEO_CALL2_REFINE, nb, 0))
                geo2_refine_flags(lvd, rec.solid, n_prop, rec.bclass, rec.refine, rec.child_map, child, d_n, ws)
                self._host_n.copy_(d_n, non_blocking=True)
                counted = torch.cuda.Event()
                counted.record()
                child_maps.append(rec.child_map)
                empty = torch.empty((0, 2), dtype=torch.int32, device=dev)
                ahead = row_bins(L + 1, make_level2(n0, L + 1, empty, child_maps))
                counted.synchronize()
                nchild = int(self._host_n[0])
                bcoord = child[:nchild]
            out.levels.append(rec)
        if with_links:
            rec = out.levels[-1]
            lvd = make_level2(n0, lf, rec.bcoord, child_maps)
            nb = lvd.nblocks
            bkey = ("links", lf)
            bcap = self.caps.get(bkey, max(1024, 8 * edges.shape[0]))
            links, _, lval = self._bins(mesh, lvd, GEO_BINS_LINKS, nb, bcap, cnt(2 * lf + 1))
            lkey = ("links_table", lf)
            cap = self.caps.get(lkey, max(1024, 2 * nb))
            cell = torch.empty(cap, dtype=torch.int32, device=dev)
            dr = torch.empty(cap, dtype=torch.uint8, device=dev)
            q = torch.empty(cap, dtype=torch.float32, device=dev)
            edge = torch.empty(cap, dtype=torch.int32, device=dev)
            geo2_cutlinks(mesh, lvd, rows, links, cap, cnt(2 * lf + 2), cell, dr, q, edge,
                          self._workspace(geo_workspace_size(GEO_CALL2_CUTLINKS, nb, 0)))
            lk = Links2D(cell, dr, q, edge)
            out.links = lk
            checks.append((2 * lf + 1, bcap, bkey, lambda c: None))

            def _apply(c):
                lk.cell, lk.dir, lk.q, lk.edge = cell[:c], dr[:c], q[:c], edge[:c]
            checks.append((2 * lf + 2, cap, lkey, _apply))
        counts = ctr.cpu().tolist()
        ok = True
        for i, cap, key, _ in checks:
            if counts[i] > cap:
                self.caps[key] = int(counts[i] * 1.1) + 1024
                ok = False
            else:
                self.caps[key] = cap
        if not ok:
            return None
        for i, cap, key, apply in checks:
            apply(counts[i])
        return out


def embed2d(verts, edges, n0, lf, d_spec=2.0, with_links=True) -> Embedding2D:
    return Embedder2D(verts.device).embed(verts, edges, n0, lf, d_spec, with_links)
