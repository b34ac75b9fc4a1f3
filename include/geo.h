/*
 * libgeo: MI355X (gfx950) geometry embedding into a block-structured forest
 * of octrees -- solid voxelization, near-wall refinement flags, and the
 * cut-link (q) lookup table for interpolated bounce-back, with the q backward.
 *
 * The operations follow the paper "GPU-native Embedding of Complex Geometries
 * in Adaptive Octree Grids Applied to the Lattice Boltzmann Method"
 * (Methodology: Spatial Binning; Voxelization and Near-Wall Refinement;
 * Boundary Cell Identification; Memory Allocations for Boundary Cells;
 * Link-Length Computation; Eq. 2 and Eq. 3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Units: base-cell units; the domain is [0,n0x] x [0,n0y] x [0,n0z].  Level
 *    L has cells of size h = 2^-L, centres at (i + 1/2) h, and blocks of 4^3
 *    cells.  A block coordinate b (level-L block units) covers cells 4b..4b+3.
 *    Cell t of a block is t = I + 4 J + 16 K (the paper's LINEAR(I, 4)).
 *  - Lattice directions: k = (cx+1) + 3 (cy+1) + 9 (cz+1), k = 13 is the rest
 *    direction; D3Q19 uses the 18 k with |c|^2 <= 2, D3Q27 the 26 k != 13.
 *  - Every pointer argument named d_* or documented as "device" is device
 *    memory owned by the caller.  The library never allocates device memory;
 *    scratch comes from the caller's workspace (see geo_workspace_size).
 *  - Every call is enqueued on the given stream (a hipStream_t; NULL is the
 *    null stream) and returns without synchronising.
 *  - Return value: GEO_OK, or a negative status for arguments that fail the
 *    host-side checks (nothing is enqueued then), a too small workspace, or a
 *    HIP launch error.
 *  - Capacity overflow is reported on the device: the required number of
 *    entries is written to the given int64 device counter, entries at index
 *    >= cap are never written, and the caller re-runs with a larger buffer.
 *  - Mesh contract (Methodology, "Overview" and "Voxelization and Near-Wall
 *    Refinement"): closed, oriented with outward normals (counter-clockwise
 *    seen from outside), not self-intersecting; every vertex coordinate lies in
 *    [1/4, n0] or is 0 (then the cell-centre frame x 2^L - 1/2 of every
 *    coordinate is exact in float64).  Zero-area triangles are allowed and
 *    ignored.  A
 *    violation gives unspecified flags but never an out-of-bounds access;
 *    vertex-range violations are counted in d_stats[GEO_STAT_CONTRACT].
 *  - Results of geo_voxelize, geo_refine_flags and the integer outputs of
 *    geo_cutlinks are exact (identical to the plain definitions evaluated in
 *    exact arithmetic); link_q is within 1e-5 of the exact value.
 */
#ifndef GEO_H
#define GEO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* geo_stream_t; /* hipStream_t */

enum {
    GEO_OK = 0,
    GEO_ERR_ARG = -1,       /* host-side argument check failed; nothing enqueued */
    GEO_ERR_WORKSPACE = -2, /* workspace smaller than geo_workspace_size(...)   */
    GEO_ERR_DEVICE = -3,    /* a HIP call or kernel launch failed                */
    GEO_ERR_TOO_LARGE = -4  /* request exceeds the fixed scratch of a no-alloc call */
};

enum { GEO_F32 = 0, GEO_F64 = 1 };                 /* vertex storage type      */
enum { GEO_PREC_F64 = 0, GEO_PREC_F32_FALLBACK = 1 }; /* arithmetic form        */
enum { GEO_BINS_ROWS = 0, GEO_BINS_LINKS = 1 };    /* kind of bins             */

/* workspace query selectors */
enum {
    GEO_CALL_BINS_ROWS = 0,
    GEO_CALL_BINS_LINKS = 1,
    GEO_CALL_REFINE = 2,
    GEO_CALL_CUTLINKS = 3,
    GEO_CALL_LINKS_DENSE = 4, /* nkeys = blocks of the level, cap ignored */
    GEO_CALL2_BINS = 5,       /* 2D bins: nkeys = row lines (ROWS) or blocks (LINKS) */
    GEO_CALL2_REFINE = 6,     /* 2D refinement: nkeys = blocks                       */
    GEO_CALL2_CUTLINKS = 7,   /* 2D cut links: nkeys = blocks                        */
    GEO_CALL_BINS_ROWS_LEVELS = 8 /* ROWS bins of several levels: nkeys = the levels'
                                     lines together, cap = their capacities together */
};

/* device statistics counters (uint64 each) */
enum {
    GEO_STAT_F32_TO_F64 = 0, /* float32 sign tests left undecided by their filters:
                                rows pass re-evaluated in float64; q kernel (both
                                forms) pairs whose links the exact pass redoes   */
    GEO_STAT_EXACT = 1,      /* float64 sign tests resolved by exact arithmetic     */
    GEO_STAT_LINKS_EXACT = 2, /* links whose nearest hit was redone exactly          */
    GEO_STAT_CONTRACT = 3,   /* vertex coordinates outside the documented range     */
    GEO_STAT_STAGED = 4,     /* candidate triangles staged by the q kernel          */
    GEO_STAT_PAIRS = 5,      /* (link, candidate) pairs passing the box test        */
    GEO_STAT_TASKS = 6,      /* (64 links x 64 candidates) tasks of the q kernel     */
    GEO_STAT_T_F64 = 7,      /* float32-form hits whose parameter t was recomputed
                                in float64 (its float32 error bound exceeded the
                                share of the 1e-5 q tolerance)                    */
    GEO_NSTATS = 8
};

#define GEO_MAX_LEVELS 12
#define GEO_MAX_RES 32767 /* n0[a] * 2^level must not exceed this */

typedef struct {
    int32_t nv;          /* number of vertices                                     */
    int32_t nt;          /* number of triangles                                    */
    int32_t vdtype;      /* GEO_F32 or GEO_F64                                     */
    const void* verts;   /* device [nv][3] float or double                         */
    const int32_t* tris; /* device [nt][3] vertex indices, outward CCW             */
} geo_mesh;

/* One level of the forest.  Blocks of level 0 are all (n0/4)^3 blocks with bx
 * fastest (geo_level0_blocks); blocks of level L+1 are the children of the
 * refined blocks of level L, in parent order, octant o = ox + 2 oy + 4 oz
 * (geo_refine_flags).  child[l] (l < level) are the child maps of the coarser
 * levels: child[l][b] = index in level l+1 of the first child of block b of
 * level l, or -1; they let a kernel find any block of this level from its
 * coordinates (the paper's neighbour-children indices). */
typedef struct {
    int32_t n0[3];                        /* base cells per axis, multiples of 4 */
    int32_t level;                        /* L, 0 <= L < GEO_MAX_LEVELS          */
    int32_t nblocks;                      /* blocks on this level                */
    const int32_t* bcoord;                /* device [nblocks][3]                 */
    const int32_t* child[GEO_MAX_LEVELS]; /* device child maps of levels < L     */
} geo_level;

/* Compressed bins (CSR).  ROWS: one key per x-row line (j, k) of the level,
 * key = j + ny * k with ny = n0y 2^L (lines of the whole domain; they do not
 * read the level's blocks, so they may be built before those are known);
 * LINKS: one key per block of the level. */
typedef struct {
    int32_t kind;     /* GEO_BINS_ROWS or GEO_BINS_LINKS                          */
    int64_t nkeys;    /* ROWS: ny*nz lines; LINKS: nblocks                          */
    int32_t* off;     /* device [nkeys+1] offsets into val                          */
    int32_t* val;     /* device [cap] entries                                       */
    int64_t cap;      /* capacity of val                                            */
    int64_t* d_count; /* device int64: number of entries needed                     */
} geo_bins;

/* Bytes of workspace needed by a call (selector GEO_CALL_*), for nkeys keys
 * (ROWS: lines, LINKS/REFINE/CUTLINKS: blocks) and cap entries. */
size_t geo_workspace_size(int32_t call, int64_t nkeys, int64_t cap);

/* Eq. 3 with the block length 4 dx_L: N_prop = 1 + floor(d_spec / (4 sqrt 2)),
 * level-independent, d_spec in base cells; the floor is taken exactly. */
int32_t geo_nprop(double d_spec);

/* Fill bcoord[(n0x/4)(n0y/4)(n0z/4)][3] with the level-0 blocks, bx fastest. */
int geo_level0_blocks(const int32_t n0[3], int32_t* bcoord, geo_stream_t stream);

/*
 * Spatial binning (Methodology, "Spatial Binning"; Algorithm 2 for the
 * widened block cover).
 *
 * ROWS: for every x-row line (j, k) of level L (line point y = (j+1/2)h,
 *   z = (k+1/2)h), the list of surface events along the line, exactly:
 *     - a parity event m >= 1 (int32 >= 0) for each triangle whose closed
 *       yz-projection contains the line point after the symbolic perturbation
 *       (y, z) -> (y + e, z + e^2), where m is the number of cell centres of
 *       the line strictly left of the crossing (cells i < m see the crossing
 *       ahead on their +x ray);
 *     - a surface interval (int32 < 0: bit 31 set, lo in bits 0-14, hi in
 *       bits 15-29) of cells whose centres lie on the closed triangle.
 *   The entry order within a line is unspecified.  The arithmetic form is
 *   selected by precision; both give identical entries.
 * LINKS: for every block of the level, the ids of the triangles that overlap
 *   the block's box widened by h/2 on every side, the region reached by the
 *   links of its cells (conservative; zero-area triangles are left out).
 *
 * mesh, lv: inputs (device arrays).  out: CSR with out->nkeys as above.
 * d_stats: device uint64[GEO_NSTATS], accumulated (may be NULL).
 */
int geo_build_bins(const geo_mesh* mesh, const geo_level* lv, int32_t kind, int32_t precision,
                   geo_bins* out, uint64_t* d_stats, void* ws, size_t ws_bytes,
                   geo_stream_t stream);

/*
 * ROWS bins of levels lmin .. lmin+nlev-1 in one pass over the triangles
 * (Methodology, "Spatial Binning"; the bins are built for every level of the
 * forest, and they do not depend on the level's blocks).  out[l] receives the
 * ROWS bins of level lmin+l with the same entries per line as
 * geo_build_bins(mesh, level lmin+l, GEO_BINS_ROWS, precision, ...) gives
 * (the order within a line is unspecified in both); each triangle is read
 * once and visits its lines of every level in turn.
 *
 * n0: base cells per axis (host int32[3], multiples of 4); 0 <= lmin,
 * 1 <= nlev, lmin + nlev <= GEO_MAX_LEVELS, n0[a] 2^(lmin+nlev-1) <=
 * GEO_MAX_RES.  out: host array of nlev bins descriptors (kind GEO_BINS_ROWS,
 * nkeys = n0y 2^L n0z 2^L of their level, distinct d_count words); the sum of
 * their nkeys must stay below 2^31 - 1.  Every *d_count is written with the
 * number of entries its level needs.  The entries of every level are complete
 * only when no level's count exceeds its cap: the levels share one staging
 * array, so an overflow of one level leaves every level's val unspecified
 * (the counts stay exact); the caller then rebuilds with larger caps.
 * d_stats: as for geo_build_bins (summed over the levels).  Workspace:
 * geo_workspace_size(GEO_CALL_BINS_ROWS_LEVELS, sum of the levels' nkeys,
 * sum of their caps).  Returns GEO_ERR_ARG or GEO_ERR_WORKSPACE with nothing
 * enqueued when an argument is out of range.
 */
int geo_build_row_bins_levels(const geo_mesh* mesh, const int32_t n0[3], int32_t lmin, int32_t nlev,
                              int32_t precision, const geo_bins* out, uint64_t* d_stats, void* ws,
                              size_t ws_bytes, geo_stream_t stream);

/*
 * Solid voxelization of level L (Methodology, "Partial Surface Voxelization"
 * and "External Cell Flag Propagation"; the result is the cell-centre
 * membership in the closed solid that those steps approximate): solid[b] bit t
 * is set iff the centre of cell t of block b lies in the closed solid bounded
 * by the mesh.  rows: ROWS bins of the same level.  solid: device
 * uint64[nblocks].  Integer work only.
 */
int geo_voxelize(const geo_level* lv, const geo_bins* rows, uint64_t* solid, geo_stream_t stream);

/*
 * Refinement flagging (Methodology, "Refinement Flagging and Propagation",
 * Eq. 3): block classes, refinement marks and the children of level L+1.
 *   bclass[b]: 0 fluid, 1 solid (>= 1 solid cell), 2 solid-boundary (solid
 *     with a fully fluid neighbour block), 3 solid-adjacent (fluid block next
 *     to a solid-boundary block);
 *   marks: M1 = (solid-boundary and eligible) or next to a solid-boundary
 *     block; then n_prop synchronous passes adding fluid blocks (and, in the
 *     first pass, solid blocks) next to a marked block; refine = marked and
 *     eligible, where eligible means every in-domain neighbour of the
 *     26-neighbourhood exists on this level (2:1 balance);
 *   child_map[b]: index of the first child in level L+1, or -1;
 *   child_bcoord: device [8*nblocks][3] capacity, children in parent order,
 *     octant o = ox + 2 oy + 4 oz; *d_nchild (device int64) = number written.
 */
int geo_refine_flags(const geo_level* lv, const uint64_t* solid, int32_t n_prop, uint8_t* bclass,
                     uint8_t* refine, int32_t* child_map, int32_t* child_bcoord,
                     int64_t* d_nchild, void* ws, size_t ws_bytes, geo_stream_t stream);

/*
 * Cut links of level L (Methodology, "Boundary Cell Identification", "Memory
 * Allocations for Boundary Cells", "Link-Length Computation", Eq. 2).
 *   link_mask[b*64+t] bit k (optional output, may be NULL): cell t of block b
 *     is fluid and the same-level centre x + h c_k is solid (classified from
 *     the ROWS bins, also where that centre's block does not exist; centres
 *     outside the domain are fluid);
 *   the table lists every set bit in the order (block, t, k):
 *     link_cell = b*64 + t, link_dir = k,
 *     link_q = min t in (0,1] with x + t h c_k on the surface,
 *     link_tri = a triangle attaining it: the smallest index among the
 *       triangles whose hit parameters round to the same multiple of
 *       1/(2^37 - 1) (exact ties included); at most 2^27 triangles;
 *   *d_nlinks (device int64) = number of links, exact; entries >= cap are not
 *     written.  The table's offsets are int32: with more than 2^31 - 1 links
 *     the outputs are unspecified (accesses stay in bounds) and the caller
 *     must split the level.
 * rows: ROWS bins of level L; links: LINKS bins of level L.
 */
int geo_cutlinks(const geo_mesh* mesh, const geo_level* lv, const geo_bins* rows,
                 const geo_bins* links, int32_t lattice, int32_t precision, uint32_t* link_mask,
                 int64_t cap, int64_t* d_nlinks, int32_t* link_cell, uint8_t* link_dir,
                 float* link_q, int32_t* link_tri, uint64_t* d_stats, void* ws, size_t ws_bytes,
                 geo_stream_t stream);

/*
 * geo_cutlinks without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, outputs, order and error behaviour
 * as geo_cutlinks, minus ws / ws_bytes: the call's scratch is a fixed device
 * array of GEO_NOALLOC_SCRATCH_BYTES compiled into the library (one per GPU
 * it runs on, held until the process ends).  The call allocates and frees
 * nothing.  It returns GEO_ERR_TOO_LARGE, before any device call and with
 * nothing enqueued, when geo_workspace_size(GEO_CALL_CUTLINKS, nblocks, cap)
 * exceeds GEO_NOALLOC_SCRATCH_BYTES.  Every call on one GPU shares that GPU's
 * scratch, which keeps the previous call's contents (each call initialises
 * what it reads): calls that overlap on one GPU (other streams, other host
 * threads) race and give unspecified results; serialise them.
 */
#define GEO_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int geo_cutlinks_noalloc(const geo_mesh* mesh, const geo_level* lv, const geo_bins* rows,
                         const geo_bins* links, int32_t lattice, int32_t precision, uint32_t* link_mask,
                         int64_t cap, int64_t* d_nlinks, int32_t* link_cell, uint8_t* link_dir,
                         float* link_q, int32_t* link_tri, uint64_t* d_stats, geo_stream_t stream);

/*
 * Dense per-block layout of a cut-link table (Methodology, "Memory
 * Allocations for Boundary Cells"): the layout a block-structured solver
 * reads.  A boundary block is a block of the level with at least one link.
 *   block_map[b] (device int32[nblocks], written): index of block b among the
 *     boundary blocks in block order, or -1;
 *   dense_q[(j * Q + s) * 64 + t] (device float[cap * Q * 64], written): q of
 *     the link of cell t of the j-th boundary block in the s-th direction of
 *     the lattice (Q = 18 for D3Q19, 26 for D3Q27; directions in increasing k,
 *     the rest direction left out), -1 where that cell has no link there;
 *   dense_tri: same layout, int32, the hit triangle (the face whose boundary
 *     condition applies), -1 where there is no link;
 *   *d_nbnd (device int64) = number of boundary blocks; boundary blocks with
 *     index >= cap are mapped but their entries are not written.
 * The link arrays are a table of geo_cutlinks, sorted by block as
 * geo_cutlinks writes it (another order gives unspecified entries, never an
 * access out of bounds).  dense_q and dense_tri must be 16-byte aligned.
 * Workspace: geo_workspace_size(GEO_CALL_LINKS_DENSE, nblocks, 0).
 */
int geo_links_dense(const geo_level* lv, int64_t n_links, const int32_t* link_cell,
                    const uint8_t* link_dir, const float* link_q, const int32_t* link_tri,
                    int32_t lattice, int64_t cap, int32_t* block_map, float* dense_q,
                    int32_t* dense_tri, int64_t* d_nbnd, void* ws, size_t ws_bytes,
                    geo_stream_t stream);

/*
 * Linear interpolated bounce-back of Bouzidi et al. (Related Work: the
 * boundary condition the link lengths serve; it needs one fluid node besides
 * the boundary node in each linked direction), applied on one level from the
 * dense layout of geo_links_dense: the boundary step of a lattice Boltzmann
 * solver.  The geometry is at rest.
 *   f_post, f_new (device, dtype GEO_F32 or GEO_F64, [nblocks][Qf][64],
 *     Qf = 19 or 27): post-collision and streamed populations;
 *     f[(b * Qf + s) * 64 + t] is cell t of block b in the s-th direction of
 *     the lattice, directions in increasing k with the rest direction
 *     included.  They must not overlap.
 *   For each link of cell x (cell t of block b) in direction p with length
 *   fraction q (from dense_q), pb = 26 - p the opposite direction, the entry
 *   of x in direction pb of f_new is set to
 *     interpolate = 0:  f*_p(x)                                  (bounce-back)
 *     q <  1/2:         2q f*_p(x) + (1 - 2q) f*_p(x - c_p)
 *     q >= 1/2:         f*_p(x) / (2q) + (1 - 1/(2q)) f*_pb(x)
 *   with f* = f_post, computed in the populations' type (the decision
 *   q < 1/2 on the float32 q).  Where q < 1/2 and x - c_p is solid (solid
 *   bits of geo_voxelize) or in no block of the level, the link takes simple
 *   bounce-back, and *d_fallback (device uint64, optional, accumulated)
 *   counts those links.  No other entry of f_new is written.
 *   block_map, dense_q: from geo_links_dense on this level and lattice
 *     (lattice 19 or 27); nbnd = boundary blocks that dense_q holds (blocks
 *     mapped to an index >= nbnd are skipped).
 *   nbr: the level's neighbour table from geo_block_neighbours, or NULL
 *     (the neighbours are then found through the forest).
 */
int geo_ibb(const geo_level* lv, const uint64_t* solid, const int32_t* block_map, const float* dense_q,
            int64_t nbnd, const int32_t* nbr, int32_t lattice, int32_t interpolate, int32_t dtype,
            const void* f_post, void* f_new, uint64_t* d_fallback, geo_stream_t stream);

/*
 * The 27-neighbourhood of every block of one level: the neighbour indices a
 * block-structured solver keeps (Methodology, "GPU-based Forest-of-Octrees":
 * blocks store the indices of a full halo of neighbours).
 *   nbr[b * 27 + o] (device int32[nblocks][27], written) = index of the
 *   same-level block at offset o = (ox+1) + 3 (oy+1) + 9 (oz+1) from block b
 *   (o = 13 is b itself), -1 where the forest has no such block, -2 outside
 *   the domain.
 */
int geo_block_neighbours(const geo_level* lv, int32_t* nbr, geo_stream_t stream);

/* ------------------------------------------------------------------------
 * 2D: quadtrees (the paper's discussion of octrees holds for quadtrees in
 * 2D).  Blocks of 4x4 cells, t = I + 4J; level 0 is all (n0x/4)(n0y/4)
 * blocks, bx fastest; the children of a refined block follow in parent order,
 * o = ox + 2 oy.  The geometry is a set of closed polygons given as edges,
 * vertices double in base-cell units within [1/4, n0] (or 0); zero-length
 * edges are ignored.  A cell is solid iff its centre lies in the closed
 * region: on an edge, or with odd parity of the edges that the +x ray from
 * it crosses, the ray lifted to height y + eps (so a horizontal edge is never
 * crossed and a vertex on the ray counts once).  The lattice is D2Q9,
 * k = (cx+1) + 3 (cy+1), 4 the rest direction.  Refinement follows the rules
 * of geo_refine_flags over the 8-neighbourhood.  All integer outputs are
 * exact; q is the first crossing, |error| <= 1e-5.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t nv;            /* vertices                               */
    int32_t ne;            /* edges                                  */
    const double* verts;   /* device [nv][2]                         */
    const int32_t* edges;  /* device [ne][2] vertex indices          */
} geo2_mesh;

typedef struct {
    int32_t n0[2];                        /* base cells per axis, multiples of 4 */
    int32_t level;
    int32_t nblocks;
    const int32_t* bcoord;                /* device [nblocks][2]                 */
    const int32_t* child[GEO_MAX_LEVELS]; /* device child maps of levels < L     */
} geo2_level;

/* Fill bcoord[(n0x/4)(n0y/4)][2] with the level-0 blocks, bx fastest. */
int geo2_level0_blocks(const int32_t n0[2], int32_t* bcoord, geo_stream_t stream);

/* Bins (Spatial Binning).  ROWS: one key per row line j of the level
 * (ny = n0y 2^L keys), the edges whose closed y range holds the line's
 * centre height.  LINKS: one key per block of the level, the edges that meet
 * the block box grown by half a cell on every side (the appendix's 2D
 * line-AABB case; a conservative test, which may add edges that never hit).
 * Order within a key is unspecified; every consumer is order-independent.
 * *bins->d_count = entries needed; entries beyond bins->cap are not written.
 * Workspace: geo_workspace_size(GEO_CALL2_BINS, nkeys, 0). */
int geo2_build_bins(const geo2_mesh* mesh, const geo2_level* lv, int32_t kind, geo_bins* bins, void* ws,
                    size_t ws_bytes, geo_stream_t stream);

/* Solid voxelization of one level: solid[b] bit t (device uint16[nblocks]). */
int geo2_voxelize(const geo2_mesh* mesh, const geo2_level* lv, const geo_bins* rows, uint16_t* solid,
                  geo_stream_t stream);

/* Refinement flags of one level (Refinement Flagging and Propagation, Eq. 3,
 * over the 8-neighbourhood); bclass, refine, child_map as for
 * geo_refine_flags, child_bcoord[4 * refined][2], *d_nchild (device int64).
 * Workspace: geo_workspace_size(GEO_CALL2_REFINE, nblocks, 0). */
int geo2_refine_flags(const geo2_level* lv, const uint16_t* solid, int32_t n_prop, uint8_t* bclass,
                      uint8_t* refine, int32_t* child_map, int32_t* child_bcoord, int64_t* d_nchild, void* ws,
                      size_t ws_bytes, geo_stream_t stream);

/* Cut links of one level (Boundary Cell Identification, Link-Length
 * Computation) for D2Q9: fluid cell x, direction k, same-level centre
 * x + h c_k solid (classified from the ROWS bins, also where its block does
 * not exist; centres outside the domain are fluid).  Table order (block, t,
 * k): link_cell = 16 b + t, link_dir = k, link_q = first crossing as a
 * fraction of the link, link_edge = the crossed edge (the smallest index
 * among edges crossed at the same double-precision parameter).
 * *d_nlinks (device int64) = number of links; entries >= cap are not written.
 * Workspace: geo_workspace_size(GEO_CALL2_CUTLINKS, nblocks, 0). */
int geo2_cutlinks(const geo2_mesh* mesh, const geo2_level* lv, const geo_bins* rows, const geo_bins* links,
                  int64_t cap, int64_t* d_nlinks, int32_t* link_cell, uint8_t* link_dir, float* link_q,
                  int32_t* link_edge, void* ws, size_t ws_bytes, geo_stream_t stream);

/*
 * Solid-flag changes of moving geometry (Limitations and Future Work: when the
 * geometry moves, nodes it no longer covers become fluid and need an initial
 * state).  prev, cur (device uint64[nblocks]): two classifications of the same
 * blocks, bit t = cell t solid -- e.g. geo_voxelize of one level with the
 * ROWS bins of the previous and of the current mesh (ROWS bins depend on the
 * level only, not on its blocks, so a previous mesh's bins classify the
 * current forest).  Writes, where the pointer is not NULL,
 *   spawned[b] = prev[b] & ~cur[b]  (solid before, fluid now),
 *   covered[b] = cur[b] & ~prev[b]  (fluid before, solid now),
 * and adds their bit counts to d_counts[0] and d_counts[1] (device int64[2],
 * accumulated; required).  Output arrays may alias neither input.
 */
int geo_solid_change(int64_t nblocks, const uint64_t* prev, const uint64_t* cur, uint64_t* spawned,
                     uint64_t* covered, int64_t* d_counts, geo_stream_t stream);

/*
 * Backward of q with respect to the vertices (not in the paper): for each
 * link i with hit triangle (v0, v1, v2), barycentrics lambda of the hit point
 * and normal n, grad_verts[v_j] += grad_q[i] * lambda_j * n / (n . h c_k)
 * (float32 atomic adds; grad_verts device float[nv][3], accumulated).
 */
int geo_cutlinks_backward(const geo_mesh* mesh, const geo_level* lv, int64_t n_links,
                          const int32_t* link_cell, const uint8_t* link_dir,
                          const int32_t* link_tri, const float* grad_q, float* grad_verts,
                          geo_stream_t stream);

/*
 * Kernel timer (measurement only; it changes nothing that is computed).
 * While enabled for a kernel, every launch of that kernel is bracketed by two
 * HIP events recorded on the stream the kernel is launched on, so one
 * kernel's device time can be read inside a call that launches several.
 * geo_kernel_timer(kernel, enable) switches it on (non-zero) or off and
 * forgets unread launches.  geo_kernel_timer_read waits for the recorded
 * events and returns the summed duration in ms and the number of timed
 * launches since the timer was enabled or last read, then starts over.  At
 * most GEO_KT_MAX_LAUNCHES launches are kept between reads; later ones are
 * not timed.  Events are created on the device current at a kernel's first
 * timed launch and are kept for reuse until the process ends.  This switch
 * and its events are the library's only host-side state (process-wide,
 * guarded by a mutex).  Returns GEO_ERR_ARG for an unknown kernel or NULL
 * outputs, GEO_ERR_DEVICE if an event wait fails.
 */
enum {
    GEO_KT_ROWS = 0,       /* ROWS bins, triangle pass (count / append)          */
    GEO_KT_VOXELIZE = 1,   /* solid voxelization of one level                   */
    GEO_KT_LINKS_BINS = 2, /* LINKS bins, triangle pass (block overlap tests)    */
    GEO_KT_CUTLINKS_Q = 3, /* cut-link q kernel (nearest hit per link)          */
    GEO_KT_IBB = 4,        /* interpolated / simple bounce-back kernel          */
    GEO_KT_COUNT = 5
};
#define GEO_KT_MAX_LAUNCHES 4096
int geo_kernel_timer(int32_t kernel, int32_t enable);
int geo_kernel_timer_read(int32_t kernel, double* total_ms, int64_t* launches);

const char* geo_version(void);

#ifdef __cplusplus
}
#endif
#endif
