"""Level-by-level embedding driver on top of the C entry points.

For L = 0 .. L_f: ROWS bins and solid voxelization of level L; for L < L_f
the refinement flags produce the blocks of level L+1 (Methodology, overview:
voxelization and refinement run level by level, top-down).  On L_f the LINKS
bins and the cut-link table follow.  The host only sizes buffers: it reads
back the next level's block count and the bin / link counts (a buffer that
was too small is grown and the call repeated).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import (GEO_BINS_LINKS, GEO_BINS_ROWS, GEO_CALL_BINS_LINKS, GEO_CALL_BINS_ROWS, GEO_CALL_CUTLINKS,
               GEO_CALL_REFINE, GEO_NSTATS, GEO_PREC_F32_FALLBACK, GEO_PREC_F64, geo_build_bins, geo_cutlinks,
               geo_cutlinks_backward, geo_level0_blocks, geo_nprop, geo_refine_flags, geo_voxelize,
               geo_workspace_size, make_bins, make_level, make_mesh)

PRECISIONS = {"f64": GEO_PREC_F64, "f32": GEO_PREC_F32_FALLBACK}


@dataclass
class Level:
    level: int
    bcoord: torch.Tensor                 # int32 [nb, 3]
    rows_off: torch.Tensor = None        # int32 [ny*nz + 1]
    rows_val: torch.Tensor = None        # int32 [n]
    solid: torch.Tensor = None           # int64 [nb] (bit t = cell t)
    bclass: torch.Tensor = None          # uint8 [nb]
    refine: torch.Tensor = None          # uint8 [nb]
    child_map: torch.Tensor = None       # int32 [nb]


@dataclass
class Links:
    mask: torch.Tensor                   # int32 [nb*64] (uint32 bits), or None
    cell: torch.Tensor                   # int32 [n]
    dir: torch.Tensor                    # uint8 [n]
    q: torch.Tensor                      # float32 [n]
    tri: torch.Tensor                    # int32 [n]
    bins_off: torch.Tensor = None
    bins_val: torch.Tensor = None

    @property
    def n(self) -> int:
        return int(self.cell.shape[0])


@dataclass
class Embedding:
    n0: tuple
    lf: int
    lattice: int
    levels: list = field(default_factory=list)
    links: Links = None
    stats: torch.Tensor = None


class Embedder:
    """Holds the workspace and remembered capacities across calls."""

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        self.ws = torch.empty(0, dtype=torch.uint8, device=self.device)
        self.caps: dict = {}
        self.events = None   # list of (name, start_event, end_event) when timing

    # -- helpers ---------------------------------------------------------------
    def _workspace(self, nbytes: int) -> torch.Tensor:
        if self.ws.numel() < nbytes:
            self.ws = torch.empty(int(nbytes * 1.25) + 4096, dtype=torch.uint8, device=self.device)
        return self.ws

    def _timed(self, name):
        if self.events is None:
            return _NoTimer()
        return _Timer(self.events, name)

    # -- the path ----------------------------------------------------------------
    def embed(self, verts: torch.Tensor, tris: torch.Tensor, n0, lf: int, lattice: int,
              d_spec: float = 2.0, precision: str = "f32", with_links: bool = True,
              with_mask: bool = False) -> Embedding:
        dev = self.device
        prec = PRECISIONS[precision]
        mesh = make_mesh(verts, tris)
        n_prop = geo_nprop(d_spec)
        stats = torch.zeros(GEO_NSTATS, dtype=torch.int64, device=dev)
        nb0 = (n0[0] // 4) * (n0[1] // 4) * (n0[2] // 4)
        bcoord = torch.empty((nb0, 3), dtype=torch.int32, device=dev)
        geo_level0_blocks(n0, bcoord)
        out = Embedding(tuple(n0), lf, lattice)
        child_maps = []
        for L in range(lf + 1):
            lvd = make_level(n0, L, bcoord, child_maps)
            rec = Level(L, bcoord)
            nkeys = (n0[1] << L) * (n0[2] << L)
            rec.rows_off, rec.rows_val = self._bins(mesh, lvd, GEO_BINS_ROWS, prec, nkeys, stats,
                                                    ("rows", L), max(4096, 2 * mesh.nt), f"rows{L}")
            rows = make_bins(GEO_BINS_ROWS, nkeys, rec.rows_off, rec.rows_val, rec.rows_val.numel(),
                             self._count)
            rec.solid = torch.empty(lvd.nblocks, dtype=torch.int64, device=dev)
            with self._timed(f"voxelize{L}"):
                geo_voxelize(lvd, rows, rec.solid)
            if L < lf:
                nb = lvd.nblocks
                rec.bclass = torch.empty(nb, dtype=torch.uint8, device=dev)
                rec.refine = torch.empty(nb, dtype=torch.uint8, device=dev)
                rec.child_map = torch.empty(nb, dtype=torch.int32, device=dev)
                child = torch.empty((8 * nb, 3), dtype=torch.int32, device=dev)
                d_n = torch.zeros(1, dtype=torch.int64, device=dev)
                ws = self._workspace(geo_workspace_size(GEO_CALL_REFINE, nb, 0))
                with self._timed(f"refine{L}"):
                    geo_refine_flags(lvd, rec.solid, n_prop, rec.bclass, rec.refine, rec.child_map, child,
                                     d_n, ws)
                nchild = int(d_n.item())
                child_maps.append(rec.child_map)
                bcoord = child[:nchild]
            else:
                self._rows_last = rows
            out.levels.append(rec)
        if with_links:
            out.links = self._cutlinks(mesh, n0, lf, out.levels[-1], child_maps, lattice, prec, stats, with_mask)
        out.stats = stats
        return out

    def _bins(self, mesh, lvd, kind, prec, nkeys, stats, key, cap0, tname):
        dev = self.device
        off = torch.empty(nkeys + 1, dtype=torch.int32, device=dev)
        cap = self.caps.get(key, cap0)
        self._count = torch.zeros(1, dtype=torch.int64, device=dev)
        call = GEO_CALL_BINS_ROWS if kind == GEO_BINS_ROWS else GEO_CALL_BINS_LINKS
        for _ in range(3):
            val = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
            bins = make_bins(kind, nkeys, off, val, cap, self._count)
            ws = self._workspace(geo_workspace_size(call, nkeys, cap))
            with self._timed(tname):
                geo_build_bins(mesh, lvd, kind, prec, bins, stats, ws)
            need = int(self._count.item())
            if need <= cap:
                self.caps[key] = cap
                return off, val[:need]
            cap = int(need * 1.1) + 1024
        raise RuntimeError("bins capacity did not converge")

    def _cutlinks(self, mesh, n0, lf, rec, child_maps, lattice, prec, stats, with_mask):
        dev = self.device
        lvd = make_level(n0, lf, rec.bcoord, child_maps)
        nb = lvd.nblocks
        loff, lval = self._bins(mesh, lvd, GEO_BINS_LINKS, prec, nb, stats, ("links", lf),
                                max(4096, 8 * mesh.nt), "linkbins")
        links = make_bins(GEO_BINS_LINKS, nb, loff, lval, lval.numel(), self._count)
        rows = make_bins(GEO_BINS_ROWS, (n0[1] << lf) * (n0[2] << lf), rec.rows_off, rec.rows_val,
                         rec.rows_val.numel(), self._count)
        mask = torch.empty(nb * 64, dtype=torch.int32, device=dev) if with_mask else None
        d_n = torch.zeros(1, dtype=torch.int64, device=dev)
        cap = self.caps.get(("links_table", lf), max(4096, 4 * nb))
        for _ in range(3):
            ws = self._workspace(geo_workspace_size(GEO_CALL_CUTLINKS, nb, cap))
            cell = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
            dr = torch.empty(max(cap, 1), dtype=torch.uint8, device=dev)
            q = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
            tri = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
            with self._timed("cutlinks"):
                geo_cutlinks(mesh, lvd, rows, links, lattice, prec, mask, cap, d_n, cell, dr, q, tri, stats, ws)
            n = int(d_n.item())
            if n <= cap:
                self.caps[("links_table", lf)] = cap
                return Links(mask, cell[:n], dr[:n], q[:n], tri[:n], loff, lval)
            cap = int(n * 1.1) + 1024
        raise RuntimeError("link capacity did not converge")


class _NoTimer:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False


class _Timer:
    def __init__(self, events, name):
        self.events, self.name = events, name

    def __enter__(self):
        self.s = torch.cuda.Event(enable_timing=True)
        self.e = torch.cuda.Event(enable_timing=True)
        self.s.record()
        return self

    def __exit__(self, *a):
        self.e.record()
        self.events.append((self.name, self.s, self.e))
        return False


def embed(verts, tris, n0, lf, lattice, d_spec=2.0, precision="f32", with_links=True,
          with_mask=False) -> Embedding:
    return Embedder(verts.device).embed(verts, tris, n0, lf, lattice, d_spec, precision, with_links, with_mask)


# ----------------------------------------------------------------------------
# autograd: q as a differentiable function of the vertices
# ----------------------------------------------------------------------------

class CutLinkQ(torch.autograd.Function):
    """Forward returns the table's q; backward scatters dL/dq onto the
    vertices with geo_cutlinks_backward (float32 atomics).  The integer parts
    of the table (which links exist, which triangle is hit) are piecewise
    constant in the vertices and carry no gradient."""

    @staticmethod
    def forward(ctx, verts, tris, emb: Embedding, child_maps):
        ctx.save_for_backward(verts, tris)
        ctx.emb = emb
        ctx.child_maps = child_maps
        return emb.links.q.clone()

    @staticmethod
    def backward(ctx, grad_q):
        verts, tris = ctx.saved_tensors
        emb = ctx.emb
        rec = emb.levels[-1]
        lvd = make_level(emb.n0, emb.lf, rec.bcoord, ctx.child_maps)
        mesh = make_mesh(verts.detach(), tris)
        g = torch.zeros((verts.shape[0], 3), dtype=torch.float32, device=verts.device)
        L = emb.links
        geo_cutlinks_backward(mesh, lvd, L.n, L.cell, L.dir, L.tri, grad_q.contiguous().float(), g)
        return g.to(verts.dtype), None, None, None


def cut_link_q(verts, tris, emb: Embedding):
    child_maps = [lv.child_map for lv in emb.levels[:-1]]
    return CutLinkQ.apply(verts, tris, emb, child_maps)
