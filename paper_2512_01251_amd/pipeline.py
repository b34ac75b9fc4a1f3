"""Level-by-level embedding driver on top of the C entry points.

ROWS bins of levels 0 .. L_f first (one pass over the triangles; they do not
depend on the blocks); then for L = 0 .. L_f the solid voxelization of level
L, and for L < L_f the refinement flags produce the blocks of level L+1
(Methodology, overview: voxelization and refinement run level by level,
top-down).  On L_f the LINKS
bins and the cut-link table follow.  The host only sizes buffers: it waits for
the next level's block count after each refinement, and for all bin and link
counts once at the end (a pass that overflowed a buffer is redone with larger
buffers; every kernel clamps to the capacity it is given).
"""
from __future__ import annotations

import time

from dataclasses import dataclass, field

import torch

from . import (GEO_BINS_LINKS, GEO_BINS_ROWS, GEO_CALL_BINS_LINKS, GEO_CALL_BINS_ROWS, GEO_CALL_BINS_ROWS_LEVELS,
               GEO_CALL_CUTLINKS, GEO_CALL_LINKS_DENSE, GEO_CALL_REFINE, GEO_NSTATS, GEO_STAT_CONTRACT,
               GEO_PREC_F32_FALLBACK, GEO_PREC_F64, geo_bins, geo_build_bins, geo_build_row_bins_levels, geo_cutlinks,
               geo_cutlinks_backward, geo_level0_blocks, geo_links_dense, geo_nprop, geo_refine_flags,
               geo_solid_change, geo_voxelize, geo_workspace_size, make_bins, make_level, make_mesh)

PRECISIONS = {"f64": GEO_PREC_F64, "f32": GEO_PREC_F32_FALLBACK}
POLL_S = 0.05   # longest poll of a pinned count before the event's wait takes over


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
    """Holds the workspace and remembered capacities across calls.  The
    level-0 block list of a grid is built once and shared, read-only, by the
    embeddings it returns for that grid."""

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        self.ws = torch.empty(0, dtype=torch.uint8, device=self.device)
        self.caps: dict = {}                 # remembered buffer capacities
        self._level0: dict = {}              # level-0 block list of the last grid
        # pinned host word for the per-level block count (read without a
        # stream-wide wait)
        self._host_n = torch.zeros(1, dtype=torch.int64, pin_memory=self.device.type == "cuda")
        self._host_np = self._host_n.numpy()
        self._poll = self.device.type == "cuda"
        self.events = None   # list of (name, start_event, end_event) when timing

    # -- helpers ---------------------------------------------------------------
    def _workspace(self, nbytes: int) -> torch.Tensor:
        if self.ws.numel() < nbytes:
            self.ws = torch.empty(int(nbytes * 1.25) + 4096, dtype=torch.uint8, device=self.device)
        return self.ws

    def _wait_count(self, ev) -> int:
        """The count copied into the pinned host word (set to -1 before the
        copy): polled, since the copy's landing is seen sooner than the
        event's wait returns; after POLL_S without it (or once that has
        happened) the event's wait is used."""
        h = self._host_np
        if self._poll:
            t_end = time.perf_counter() + POLL_S
            while h[0] < 0:
                if time.perf_counter() > t_end:
                    self._poll = False
                    break
            if h[0] >= 0:
                return int(h[0])
        ev.synchronize()
        return int(h[0])

    def _timed(self, name):
        if self.events is None:
            return _NoTimer()
        return _Timer(self.events, name)

    # -- the path ----------------------------------------------------------------
    def embed(self, verts: torch.Tensor, tris: torch.Tensor, n0, lf: int, lattice: int,
              d_spec: float = 2.0, precision: str = "f32", with_links: bool = True,
              with_mask: bool = False, check_contract: bool = True) -> Embedding:
        """Embeds the mesh (levels 0..lf, then the cut links of level lf).
        Raises ValueError when a vertex coordinate breaks the coordinate
        range of the library (the results would be unspecified), unless
        check_contract is False; the violation count is then in stats."""
        # each pass sizes at least the first level whose buffers overflowed
        for _ in range(lf + 4):
            out = self._embed_once(verts, tris, n0, lf, lattice, d_spec, precision, with_links, with_mask,
                                   check_contract)
            if out is not None:
                return out
        raise RuntimeError("buffer capacities did not converge")

    def _embed_once(self, verts, tris, n0, lf, lattice, d_spec, precision, with_links, with_mask,
                    check_contract=True):
        """One pass over all levels.  Bin and link counts are checked once, at
        the end: every kernel clamps to the capacity it is given, so a pass that
        overflowed a buffer is memory-safe and is simply redone with larger
        buffers (None is returned).  The host waits only for the child count of
        each level (it sizes the next level) and for the final counts."""
        dev = self.device
        prec = PRECISIONS[precision]
        mesh = make_mesh(verts, tris)
        n_prop = geo_nprop(d_spec)
        # one zero-filled buffer for the statistics and every device counter
        ctr = torch.zeros(GEO_NSTATS + 2 * lf + 4, dtype=torch.int64, device=dev)
        stats = ctr[:GEO_NSTATS]
        cnt = lambda i: ctr[GEO_NSTATS + i:GEO_NSTATS + i + 1]
        checks = []   # (counter index, capacity, capacity key, apply(count))
        nb0 = (n0[0] // 4) * (n0[1] // 4) * (n0[2] // 4)
        # the level-0 blocks depend on n0 only: built once per grid and shared
        # (read-only) by the embeddings of later calls
        key0 = ("level0", tuple(int(x) for x in n0))
        bcoord = self._level0.get(key0)
        if bcoord is None:
            bcoord = torch.empty((nb0, 3), dtype=torch.int32, device=dev)
            geo_level0_blocks(n0, bcoord)
            self._level0 = {key0: bcoord}
        out = Embedding(tuple(n0), lf, lattice)
        child_maps = []
        rows = None

        # ROWS bins depend on the level, not on its blocks: those of every
        # level are built first, in one pass over the triangles
        row_bins = self._row_bins_levels(mesh, n0, lf, prec, stats, cnt)
        # Each level's voxelization is launched as soon as its block count is
        # known: the next level's descriptor and solid buffer (at the capacity
        # 8 nb) are made while the GPU refines, the rest of a level's buffers
        # after its voxelization is enqueued.
        lvd = make_level(n0, 0, bcoord, child_maps)
        solid = torch.empty(nb0, dtype=torch.int64, device=dev)
        with self._timed("voxelize0"):
            geo_voxelize(lvd, row_bins[0][5], solid)
        for L in range(lf + 1):
            nb = lvd.nblocks
            rec = Level(L, bcoord)
            rec.solid = solid
            nkeys, key, cap, rec.rows_off, val, rows = row_bins[L]
            rec.rows_val = val
            checks.append((L, cap, key, lambda c, rec=rec, val=val: setattr(rec, "rows_val", val[:c])))
            out.levels.append(rec)
            if L == lf:
                break
            rec.bclass = torch.empty(nb, dtype=torch.uint8, device=dev)
            rec.refine = torch.empty(nb, dtype=torch.uint8, device=dev)
            rec.child_map = torch.empty(nb, dtype=torch.int32, device=dev)
            child = torch.empty((8 * nb, 3), dtype=torch.int32, device=dev)
            ws = self._workspace(geo_workspace_size(GEO_CALL_REFINE, nb, 0))
            d_n = cnt(lf + 1 + L)
            with self._timed(f"refine{L}"):
                geo_refine_flags(lvd, rec.solid, n_prop, rec.bclass, rec.refine, rec.child_map, child, d_n, ws)
            self._host_np[0] = -1
            self._host_n.copy_(d_n, non_blocking=True)
            counted = torch.cuda.Event()
            counted.record()
            child_maps.append(rec.child_map)
            nxt = make_level(n0, L + 1, child, child_maps)
            solid_next = torch.empty(8 * nb, dtype=torch.int64, device=dev)
            nchild = self._wait_count(counted)
            nxt.nblocks = nchild
            with self._timed(f"voxelize{L + 1}"):
                geo_voxelize(nxt, row_bins[L + 1][5], solid_next)
            lvd, bcoord, solid = nxt, child[:nchild], solid_next[:nchild]
        if with_links:
            out.links = self._cutlinks(mesh, n0, lf, out.levels[-1], child_maps, rows, lattice, prec, stats,
                                       with_mask, cnt(2 * lf + 1), cnt(2 * lf + 2), checks)
        # the final wait: every count and statistic at once
        allc = ctr.cpu().tolist()
        if check_contract and allc[GEO_STAT_CONTRACT]:
            raise ValueError(f"{allc[GEO_STAT_CONTRACT]} vertex coordinates lie outside the library's coordinate "
                             "range (each coordinate must be 0 or in [1/4, n0], finite); the results are unspecified")
        counts = allc[GEO_NSTATS:]
        if with_links and counts[2 * lf + 2] > 2 ** 31 - 1:
            raise RuntimeError(f"{counts[2 * lf + 2]} links exceed the table's int32 offsets")
        ok = True
        for i, cap, key, apply in checks:
            if counts[i] > cap:
                self.caps[key] = int(counts[i] * 1.1) + 1024
                ok = False
            else:
                self.caps[key] = cap
        if not ok:
            return None
        for i, cap, key, apply in checks:
            apply(counts[i])
        out.stats = stats
        return out

    def _row_bins_levels(self, mesh, n0, lf, prec, stats, cnt):
        """ROWS bins of levels 0..lf with one C call: per level (nkeys,
        capacity key, capacity, off, val, descriptor); level L counts into
        cnt(L)."""
        dev = self.device
        out, bins, spans = [], [], []
        pos = 0
        for L in range(lf + 1):  # one allocation, the arrays 256-byte aligned
            nkeys = (n0[1] << L) * (n0[2] << L)
            key = ("rows", L)
            cap = self.caps.get(key, max(4096, 2 * mesh.nt))
            o = pos
            pos = (pos + nkeys + 1 + 63) // 64 * 64
            v = pos
            pos = (pos + max(cap, 1) + 63) // 64 * 64
            spans.append((nkeys, key, cap, o, v))
        buf = torch.empty(pos, dtype=torch.int32, device=dev)
        # descriptors from addresses, so that the launch does not wait for the
        # tensor views (made while the GPU runs the pass)
        base, cbase = buf.data_ptr(), cnt(0).data_ptr()
        for L, (nkeys, key, cap, o, v) in enumerate(spans):
            bins.append(geo_bins(GEO_BINS_ROWS, nkeys, base + 4 * o, base + 4 * v, cap, cbase + 8 * L))
        ws = self._workspace(geo_workspace_size(GEO_CALL_BINS_ROWS_LEVELS, sum(x[0] for x in spans),
                                                sum(x[2] for x in spans)))
        with self._timed("rows"):
            geo_build_row_bins_levels(mesh, n0, 0, prec, bins, stats, ws)
        for L, (nkeys, key, cap, o, v) in enumerate(spans):
            out.append((nkeys, key, cap, buf[o:o + nkeys + 1], buf[v:v + max(cap, 1)], bins[L]))
        return out

    def _bins(self, mesh, lvd, kind, prec, nkeys, stats, cap, d_count, tname):
        dev = self.device
        off = torch.empty(nkeys + 1, dtype=torch.int32, device=dev)
        val = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        bins = make_bins(kind, nkeys, off, val, cap, d_count)
        call = GEO_CALL_BINS_ROWS if kind == GEO_BINS_ROWS else GEO_CALL_BINS_LINKS
        ws = self._workspace(geo_workspace_size(call, nkeys, cap))
        with self._timed(tname):
            geo_build_bins(mesh, lvd, kind, prec, bins, stats, ws)
        return off, val

    def _cutlinks(self, mesh, n0, lf, rec, child_maps, rows, lattice, prec, stats, with_mask, d_bins, d_n,
                  checks):
        dev = self.device
        lvd = make_level(n0, lf, rec.bcoord, child_maps)
        nb = lvd.nblocks
        key = ("links", lf)
        bcap = self.caps.get(key, max(4096, 8 * mesh.nt))
        # no statistics: the vertex contract was counted by the ROWS call, and
        # the LINKS pass keeps no other counter
        loff, lval = self._bins(mesh, lvd, GEO_BINS_LINKS, prec, nb, None, bcap, d_bins, "linkbins")
        links = make_bins(GEO_BINS_LINKS, nb, loff, lval, bcap, d_bins)
        mask = torch.empty(nb * 64, dtype=torch.int32, device=dev) if with_mask else None
        lkey = ("links_table", lf)
        cap = self.caps.get(lkey, max(4096, 4 * nb))
        ws = self._workspace(geo_workspace_size(GEO_CALL_CUTLINKS, nb, cap))
        cell = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        dr = torch.empty(max(cap, 1), dtype=torch.uint8, device=dev)
        q = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
        tri = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        with self._timed("cutlinks"):
            geo_cutlinks(mesh, lvd, rows, links, lattice, prec, mask, cap, d_n, cell, dr, q, tri, stats, ws)
        L = Links(mask, cell, dr, q, tri, loff, lval)
        checks.append((2 * lf + 1, bcap, key, lambda c: setattr(L, "bins_val", lval[:c])))

        def _apply(c):
            L.cell, L.dir, L.q, L.tri = cell[:c], dr[:c], q[:c], tri[:c]
        checks.append((2 * lf + 2, cap, lkey, _apply))
        return L


@dataclass
class DenseLinks:
    """Dense per-block layout of a link table: block_map [nb] (-1 or the
    boundary-block index), q and tri [nbnd, Q, 64] (-1 where no link)."""
    block_map: torch.Tensor
    q: torch.Tensor
    tri: torch.Tensor

    @property
    def nbnd(self) -> int:
        return int(self.q.shape[0])


def links_dense(emb: "Embedding", caps: dict = None) -> DenseLinks:
    """The paper's dense link-length layout built from the table of emb."""
    rec, L = emb.levels[-1], emb.links
    dev = L.cell.device
    nb = int(rec.bcoord.shape[0])
    qd = 26 if emb.lattice == 27 else 18
    lvd = make_level(emb.n0, emb.lf, rec.bcoord, [lv.child_map for lv in emb.levels[:-1]])
    caps = {} if caps is None else caps
    cap = caps.get("dense", max(64, nb // 4))
    ws = torch.empty(geo_workspace_size(GEO_CALL_LINKS_DENSE, nb, 0), dtype=torch.uint8, device=dev)
    block_map = torch.empty(max(nb, 1), dtype=torch.int32, device=dev)
    d_n = torch.zeros(1, dtype=torch.int64, device=dev)
    for _ in range(2):
        q = torch.empty((cap, qd, 64), dtype=torch.float32, device=dev)
        tri = torch.empty((cap, qd, 64), dtype=torch.int32, device=dev)
        geo_links_dense(lvd, L.n, L.cell, L.dir, L.q, L.tri, emb.lattice, cap, block_map, q, tri, d_n, ws)
        n = int(d_n.item())
        if n <= cap:
            caps["dense"] = cap
            return DenseLinks(block_map[:nb], q[:n], tri[:n])
        cap = n
    raise RuntimeError("dense layout capacity did not converge")


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


# ----------------------------------------------------------------------------
# moving geometry: per-step rebuild, solid changes, gradient
# ----------------------------------------------------------------------------

@dataclass
class SolidChange:
    """Cells of one level whose solid flag changed since the previous
    geometry: bit t of spawned[b] (covered[b]) is set iff cell t of block b
    was solid (fluid) under the previous mesh and is fluid (solid) now;
    counts = [spawned, covered] on the device."""
    level: int
    spawned: torch.Tensor
    covered: torch.Tensor
    counts: torch.Tensor


def solid_change(prev: Embedding, emb: Embedding, level: int = None) -> SolidChange:
    """Solid changes on one level (default: the finest) of emb against the
    geometry that prev embedded on the same grid.  The previous mesh
    classifies the current forest through its ROWS bins of that level, which
    depend on the level and not on its blocks.  No host wait."""
    L = emb.lf if level is None else level
    if tuple(prev.n0) != tuple(emb.n0) or L >= len(prev.levels):
        raise ValueError("solid_change needs two embeddings of the same grid and level")
    rec, old = emb.levels[L], prev.levels[L]
    dev = rec.bcoord.device
    nb = int(rec.bcoord.shape[0])
    lvd = make_level(emb.n0, L, rec.bcoord, [lv.child_map for lv in emb.levels[:L]])
    nkeys = (emb.n0[1] << L) * (emb.n0[2] << L)
    n_old = int(old.rows_val.numel())
    d_cnt = torch.full((1,), n_old, dtype=torch.int64, device=dev)
    rows = make_bins(GEO_BINS_ROWS, nkeys, old.rows_off, old.rows_val, n_old, d_cnt)
    before = torch.empty(nb, dtype=torch.int64, device=dev)
    geo_voxelize(lvd, rows, before)
    spawned = torch.empty(nb, dtype=torch.int64, device=dev)
    covered = torch.empty(nb, dtype=torch.int64, device=dev)
    counts = torch.zeros(2, dtype=torch.int64, device=dev)
    geo_solid_change(nb, before, rec.solid, spawned, covered, counts)
    return SolidChange(L, spawned, covered, counts)


def shape_step(embedder: Embedder, verts: torch.Tensor, tris: torch.Tensor, n0, lf: int, lattice: int,
               d_spec: float = 2.0, precision: str = "f32", prev: Embedding = None):
    """One step of a shape-sensitivity loop over a moving geometry: rebuild
    the embedding for the current vertices (every level re-binned), the
    cut-link lengths q as a differentiable function of the vertices, and the
    solid changes of the finest level against the previous step's embedding
    (None on the first step).  Returns (emb, q, change)."""
    emb = embedder.embed(verts.detach(), tris, n0, lf, lattice, d_spec, precision, True)
    q = cut_link_q(verts, tris, emb)
    change = solid_change(prev, emb) if prev is not None else None
    return emb, q, change
