"""MI355X (gfx950) geometry embedding into a block-structured forest of octrees.

Thin ctypes binding of libgeo.so (include/geo.h): the functions below carry
the C names and only marshal arguments; every step of the path runs in the
HIP kernels of the library.  torch supplies device memory and streams.

The library must have been built (paper_2512_01251_amd/build_lib.py); there is
no fallback: importing the binding fails loudly when libgeo.so is missing.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgeo.so")

GEO_OK, GEO_ERR_ARG, GEO_ERR_WORKSPACE, GEO_ERR_DEVICE, GEO_ERR_TOO_LARGE = 0, -1, -2, -3, -4
GEO_NOALLOC_SCRATCH_BYTES = 64 << 20
GEO_F32, GEO_F64 = 0, 1
GEO_PREC_F64, GEO_PREC_F32_FALLBACK = 0, 1
GEO_BINS_ROWS, GEO_BINS_LINKS = 0, 1
GEO_CALL_BINS_ROWS, GEO_CALL_BINS_LINKS, GEO_CALL_REFINE, GEO_CALL_CUTLINKS, GEO_CALL_LINKS_DENSE = 0, 1, 2, 3, 4
GEO_CALL2_BINS, GEO_CALL2_REFINE, GEO_CALL2_CUTLINKS = 5, 6, 7
GEO_CALL_BINS_ROWS_LEVELS = 8
GEO_STAT_F32_TO_F64, GEO_STAT_EXACT, GEO_STAT_LINKS_EXACT, GEO_STAT_CONTRACT, GEO_STAT_STAGED, GEO_STAT_PAIRS = 0, 1, 2, 3, 4, 5
GEO_STAT_TASKS, GEO_STAT_T_F64 = 6, 7
GEO_NSTATS = 8
GEO_KT_ROWS, GEO_KT_VOXELIZE, GEO_KT_LINKS_BINS, GEO_KT_CUTLINKS_Q, GEO_KT_IBB, GEO_KT_COUNT = 0, 1, 2, 3, 4, 5
GEO_KT_MAX_LAUNCHES = 4096
GEO_MAX_LEVELS = 12
GEO_MAX_RES = 32767

EXPORTS = ["geo_workspace_size", "geo_nprop", "geo_level0_blocks", "geo_build_bins", "geo_build_row_bins_levels", "geo_voxelize",
           "geo_refine_flags", "geo_cutlinks", "geo_cutlinks_noalloc", "geo_cutlinks_backward", "geo_links_dense", "geo_ibb", "geo_block_neighbours", "geo_solid_change", "geo2_level0_blocks", "geo2_build_bins",
           "geo2_voxelize", "geo2_refine_flags", "geo2_cutlinks", "geo_kernel_timer", "geo_kernel_timer_read", "geo_version"]


class GeoError(RuntimeError):
    pass


class geo_mesh(C.Structure):
    _fields_ = [("nv", C.c_int32), ("nt", C.c_int32), ("vdtype", C.c_int32),
                ("verts", C.c_void_p), ("tris", C.c_void_p)]


class geo_level(C.Structure):
    _fields_ = [("n0", C.c_int32 * 3), ("level", C.c_int32), ("nblocks", C.c_int32),
                ("bcoord", C.c_void_p), ("child", C.c_void_p * GEO_MAX_LEVELS)]


class geo2_mesh(C.Structure):
    _fields_ = [("nv", C.c_int32), ("ne", C.c_int32), ("verts", C.c_void_p), ("edges", C.c_void_p)]


class geo2_level(C.Structure):
    _fields_ = [("n0", C.c_int32 * 2), ("level", C.c_int32), ("nblocks", C.c_int32),
                ("bcoord", C.c_void_p), ("child", C.c_void_p * GEO_MAX_LEVELS)]


class geo_bins(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nkeys", C.c_int64), ("off", C.c_void_p), ("val", C.c_void_p),
                ("cap", C.c_int64), ("d_count", C.c_void_p)]


_lib = None


def lib():
    """Load libgeo.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise GeoError(f"{LIB_PATH} not found: build it with paper_2512_01251_amd/build_lib.py")
        L = C.CDLL(LIB_PATH)
        P, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        MP, LP, BP = C.POINTER(geo_mesh), C.POINTER(geo_level), C.POINTER(geo_bins)
        L.geo_workspace_size.argtypes = [i32, i64, i64]
        L.geo_workspace_size.restype = sz
        L.geo_nprop.argtypes = [C.c_double]
        L.geo_nprop.restype = i32
        L.geo_level0_blocks.argtypes = [P, P, P]
        L.geo_build_bins.argtypes = [MP, LP, i32, i32, BP, P, P, sz, P]
        L.geo_build_row_bins_levels.argtypes = [MP, C.POINTER(C.c_int32), i32, i32, i32, BP, P, P, sz, P]
        L.geo_voxelize.argtypes = [LP, BP, P, P]
        L.geo_refine_flags.argtypes = [LP, P, i32, P, P, P, P, P, P, sz, P]
        L.geo_cutlinks.argtypes = [MP, LP, BP, BP, i32, i32, P, i64, P, P, P, P, P, P, P, sz, P]
        L.geo_cutlinks_noalloc.argtypes = [MP, LP, BP, BP, i32, i32, P, i64, P, P, P, P, P, P, P]
        L.geo_cutlinks_backward.argtypes = [MP, LP, i64, P, P, P, P, P, P]
        L.geo_links_dense.argtypes = [LP, i64, P, P, P, P, i32, i64, P, P, P, P, P, sz, P]
        L.geo_ibb.argtypes = [LP, P, P, P, i64, P, i32, i32, i32, P, P, P, P]
        L.geo_block_neighbours.argtypes = [LP, P, P]
        L.geo_solid_change.argtypes = [i64, P, P, P, P, P, P]
        M2, L2 = C.POINTER(geo2_mesh), C.POINTER(geo2_level)
        L.geo2_level0_blocks.argtypes = [P, P, P]
        L.geo2_build_bins.argtypes = [M2, L2, i32, BP, P, sz, P]
        L.geo2_voxelize.argtypes = [M2, L2, BP, P, P]
        L.geo2_refine_flags.argtypes = [L2, P, i32, P, P, P, P, P, P, sz, P]
        L.geo2_cutlinks.argtypes = [M2, L2, BP, BP, i64, P, P, P, P, P, P, sz, P]
        L.geo_kernel_timer.argtypes = [i32, i32]
        L.geo_kernel_timer_read.argtypes = [i32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.geo_version.restype = C.c_char_p
        for name in EXPORTS:
            getattr(L, name).restype = getattr(L, name).restype or C.c_int
        _lib = L
    return _lib


_STATUS = {GEO_ERR_ARG: "invalid argument", GEO_ERR_WORKSPACE: "workspace too small",
           GEO_ERR_DEVICE: "HIP call or launch failed",
           GEO_ERR_TOO_LARGE: f"request exceeds the {GEO_NOALLOC_SCRATCH_BYTES >> 20} MiB scratch of a no-alloc call"}


def _check(rc: int, what: str):
    if rc != GEO_OK:
        raise GeoError(f"{what} failed with status {rc} ({_STATUS.get(rc, 'unknown status')})")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:  # the current stream of the current device
        import torch
        return C.c_void_p(torch._C._cuda_getCurrentRawStream(torch.cuda.current_device()))
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


# ----------------------------------------------------------------------------
# descriptor constructors (torch tensors -> C structs)
# ----------------------------------------------------------------------------

def make_mesh(verts, tris) -> geo_mesh:
    import torch
    assert verts.is_cuda and tris.is_cuda and verts.is_contiguous() and tris.is_contiguous()
    assert tris.dtype == torch.int32 and verts.dtype in (torch.float32, torch.float64)
    return geo_mesh(verts.shape[0], tris.shape[0], GEO_F64 if verts.dtype == torch.float64 else GEO_F32,
                    verts.data_ptr(), tris.data_ptr())


def make_level(n0, level: int, bcoord, child_maps) -> geo_level:
    lv = geo_level()
    for a in range(3):
        lv.n0[a] = int(n0[a])
    lv.level = level
    lv.nblocks = int(bcoord.shape[0])
    lv.bcoord = bcoord.data_ptr() if bcoord.numel() else None
    for l in range(level):
        lv.child[l] = child_maps[l].data_ptr()
    return lv


def make_mesh2(verts, edges) -> geo2_mesh:
    import torch
    assert verts.is_cuda and edges.is_cuda and verts.is_contiguous() and edges.is_contiguous()
    assert verts.dtype == torch.float64 and edges.dtype == torch.int32
    return geo2_mesh(verts.shape[0], edges.shape[0], verts.data_ptr(), edges.data_ptr())


def make_level2(n0, level: int, bcoord, child_maps) -> geo2_level:
    lv = geo2_level()
    for a in range(2):
        lv.n0[a] = int(n0[a])
    lv.level = level
    lv.nblocks = int(bcoord.shape[0])
    lv.bcoord = bcoord.data_ptr() if bcoord.numel() else None
    for l in range(level):
        lv.child[l] = child_maps[l].data_ptr()
    return lv


def make_bins(kind: int, nkeys: int, off, val, cap: int, d_count) -> geo_bins:
    return geo_bins(kind, nkeys, off.data_ptr(), val.data_ptr() if val.numel() else None, cap,
                    d_count.data_ptr())


# ----------------------------------------------------------------------------
# the C entry points (argument marshalling only)
# ----------------------------------------------------------------------------

def geo_workspace_size(call: int, nkeys: int, cap: int) -> int:
    return int(lib().geo_workspace_size(call, nkeys, cap))


def geo_nprop(d_spec: float) -> int:
    return int(lib().geo_nprop(float(d_spec)))


def geo_version() -> str:
    return lib().geo_version().decode()


def geo_kernel_timer(kernel: int, enable: bool):
    _check(lib().geo_kernel_timer(int(kernel), 1 if enable else 0), "geo_kernel_timer")


def geo_kernel_timer_read(kernel: int):
    """(summed duration in ms, number of timed launches) since the last read."""
    ms, n = C.c_double(0.0), C.c_int64(0)
    _check(lib().geo_kernel_timer_read(int(kernel), C.byref(ms), C.byref(n)), "geo_kernel_timer_read")
    return ms.value, n.value


def geo_level0_blocks(n0, bcoord, stream=None):
    arr = (C.c_int32 * 3)(*[int(x) for x in n0])
    _check(lib().geo_level0_blocks(arr, _ptr(bcoord), _stream(stream)), "geo_level0_blocks")


def geo_build_bins(mesh: geo_mesh, level: geo_level, kind: int, precision: int, bins: geo_bins,
                   stats, ws, stream=None):
    rc = lib().geo_build_bins(C.byref(mesh), C.byref(level), kind, precision, C.byref(bins),
                              _ptr(stats), _ptr(ws), ws.numel() if ws is not None else 0,
                              _stream(stream))
    _check(rc, "geo_build_bins")


def geo_build_row_bins_levels(mesh: geo_mesh, n0, lmin: int, precision: int, bins, stats, ws, stream=None):
    """ROWS bins of levels lmin .. lmin+len(bins)-1 in one call; bins: a
    sequence of geo_bins, one per level."""
    n = len(bins)
    arr = (geo_bins * max(n, 1))(*bins)
    n0c = (C.c_int32 * 3)(*[int(x) for x in n0])
    rc = lib().geo_build_row_bins_levels(C.byref(mesh), n0c, lmin, n, precision, arr, _ptr(stats), _ptr(ws),
                                         ws.numel() if ws is not None else 0, _stream(stream))
    _check(rc, "geo_build_row_bins_levels")


def geo_voxelize(level: geo_level, rows: geo_bins, solid, stream=None):
    _check(lib().geo_voxelize(C.byref(level), C.byref(rows), _ptr(solid), _stream(stream)),
           "geo_voxelize")


def geo_refine_flags(level: geo_level, solid, n_prop: int, bclass, refine, child_map, child_bcoord,
                     d_nchild, ws, stream=None):
    rc = lib().geo_refine_flags(C.byref(level), _ptr(solid), int(n_prop), _ptr(bclass), _ptr(refine),
                                _ptr(child_map), _ptr(child_bcoord), _ptr(d_nchild), _ptr(ws),
                                ws.numel() if ws is not None else 0, _stream(stream))
    _check(rc, "geo_refine_flags")


def geo_cutlinks(mesh: geo_mesh, level: geo_level, rows: geo_bins, links: geo_bins, lattice: int,
                 precision: int, link_mask, cap: int, d_nlinks, link_cell, link_dir, link_q,
                 link_tri, stats, ws, stream=None):
    rc = lib().geo_cutlinks(C.byref(mesh), C.byref(level), C.byref(rows), C.byref(links), int(lattice),
                            int(precision), _ptr(link_mask), int(cap), _ptr(d_nlinks), _ptr(link_cell),
                            _ptr(link_dir), _ptr(link_q), _ptr(link_tri), _ptr(stats), _ptr(ws),
                            ws.numel() if ws is not None else 0, _stream(stream))
    _check(rc, "geo_cutlinks")


def geo_cutlinks_noalloc(mesh: geo_mesh, level: geo_level, rows: geo_bins, links: geo_bins, lattice: int,
                         precision: int, link_mask, cap: int, d_nlinks, link_cell, link_dir, link_q, link_tri,
                         stats, stream=None):
    rc = lib().geo_cutlinks_noalloc(C.byref(mesh), C.byref(level), C.byref(rows), C.byref(links), int(lattice),
                                    int(precision), _ptr(link_mask), int(cap), _ptr(d_nlinks), _ptr(link_cell),
                                    _ptr(link_dir), _ptr(link_q), _ptr(link_tri), _ptr(stats), _stream(stream))
    _check(rc, "geo_cutlinks_noalloc")


def geo_links_dense(level: geo_level, n_links: int, link_cell, link_dir, link_q, link_tri, lattice: int,
                    cap: int, block_map, dense_q, dense_tri, d_nbnd, ws, stream=None):
    rc = lib().geo_links_dense(C.byref(level), int(n_links), _ptr(link_cell), _ptr(link_dir), _ptr(link_q),
                               _ptr(link_tri), int(lattice), int(cap), _ptr(block_map), _ptr(dense_q),
                               _ptr(dense_tri), _ptr(d_nbnd), _ptr(ws), ws.numel() if ws is not None else 0,
                               _stream(stream))
    _check(rc, "geo_links_dense")


def geo_block_neighbours(level: geo_level, nbr, stream=None):
    _check(lib().geo_block_neighbours(C.byref(level), _ptr(nbr), _stream(stream)), "geo_block_neighbours")


def geo_ibb(level: geo_level, solid, block_map, dense_q, nbnd: int, lattice: int, interpolate: bool, f_post,
            f_new, d_fallback=None, stream=None, nbr=None):
    import torch
    if f_post.dtype != f_new.dtype or f_post.dtype not in (torch.float32, torch.float64):
        raise GeoError("geo_ibb: f_post and f_new must both be float32 or both float64")
    dt = GEO_F64 if f_post.dtype == torch.float64 else GEO_F32
    rc = lib().geo_ibb(C.byref(level), _ptr(solid), _ptr(block_map), _ptr(dense_q), int(nbnd), _ptr(nbr),
                       int(lattice), int(bool(interpolate)), dt, _ptr(f_post), _ptr(f_new), _ptr(d_fallback),
                       _stream(stream))
    _check(rc, "geo_ibb")


def geo_solid_change(nblocks: int, prev, cur, spawned, covered, d_counts, stream=None):
    rc = lib().geo_solid_change(int(nblocks), _ptr(prev), _ptr(cur), _ptr(spawned), _ptr(covered), _ptr(d_counts),
                                _stream(stream))
    _check(rc, "geo_solid_change")


def geo2_level0_blocks(n0, bcoord, stream=None):
    arr = (C.c_int32 * 2)(*[int(x) for x in n0])
    _check(lib().geo2_level0_blocks(arr, _ptr(bcoord), _stream(stream)), "geo2_level0_blocks")


def geo2_build_bins(mesh: geo2_mesh, level: geo2_level, kind: int, bins: geo_bins, ws, stream=None):
    _check(lib().geo2_build_bins(C.byref(mesh), C.byref(level), int(kind), C.byref(bins), _ptr(ws),
                                 ws.numel() if ws is not None else 0, _stream(stream)), "geo2_build_bins")


def geo2_voxelize(mesh: geo2_mesh, level: geo2_level, rows: geo_bins, solid, stream=None):
    _check(lib().geo2_voxelize(C.byref(mesh), C.byref(level), C.byref(rows), _ptr(solid), _stream(stream)),
           "geo2_voxelize")


def geo2_refine_flags(level: geo2_level, solid, n_prop: int, bclass, refine, child_map, child_bcoord, d_nchild, ws,
                      stream=None):
    _check(lib().geo2_refine_flags(C.byref(level), _ptr(solid), int(n_prop), _ptr(bclass), _ptr(refine),
                                   _ptr(child_map), _ptr(child_bcoord), _ptr(d_nchild), _ptr(ws),
                                   ws.numel() if ws is not None else 0, _stream(stream)), "geo2_refine_flags")


def geo2_cutlinks(mesh: geo2_mesh, level: geo2_level, rows: geo_bins, links: geo_bins, cap: int, d_nlinks,
                  link_cell, link_dir, link_q, link_edge, ws, stream=None):
    _check(lib().geo2_cutlinks(C.byref(mesh), C.byref(level), C.byref(rows), C.byref(links), int(cap),
                               _ptr(d_nlinks), _ptr(link_cell), _ptr(link_dir), _ptr(link_q), _ptr(link_edge),
                               _ptr(ws), ws.numel() if ws is not None else 0, _stream(stream)), "geo2_cutlinks")


def geo_cutlinks_backward(mesh: geo_mesh, level: geo_level, n_links: int, link_cell, link_dir,
                          link_tri, grad_q, grad_verts, stream=None):
    rc = lib().geo_cutlinks_backward(C.byref(mesh), C.byref(level), int(n_links), _ptr(link_cell),
                                     _ptr(link_dir), _ptr(link_tri), _ptr(grad_q), _ptr(grad_verts),
                                     _stream(stream))
    _check(rc, "geo_cutlinks_backward")
