// C-ABI entry points of libgeo: host-side argument checks, workspace
// partitioning and kernel launches (declared in include/geo.h).
#include <math.h>

#include "geo_internal.h"

size_t geo_refine_ws_bytes(int64_t nb);
size_t geo_cutlinks_ws_bytes(int64_t nb, int64_t cap);

namespace {

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

size_t bins_ws_bytes(int64_t nkeys, int64_t cap) {
    const size_t c = (size_t)(cap > 0 ? cap : 0);
    return al(sizeof(int2) * c) + al(sizeof(int32_t) * c) + al(sizeof(int32_t) * ((size_t)nkeys + 1)) +
           al(geo_scan_partials_bytes(nkeys));
}

size_t rows_levels_ws_bytes(int64_t nkeys, int64_t cap) { return bins_ws_bytes(nkeys, cap) + al(sizeof(int64_t)); }

bool check_level(const geo_level* lv) {
    if (!lv) return false;
    if (lv->level < 0 || lv->level >= GEO_MAX_LEVELS || lv->nblocks < 0) return false;
    for (int a = 0; a < 3; a++) {
        if (lv->n0[a] <= 0 || lv->n0[a] % 4 != 0) return false;
        if ((int64_t)lv->n0[a] << lv->level > GEO_MAX_RES) return false;
    }
    if (lv->nblocks > 0 && !lv->bcoord) return false;
    if ((int64_t)lv->nblocks * 64 > INT32_MAX) return false;
    // the child maps are read only through the blocks of this level (a level
    // without blocks may follow one without refined blocks)
    if (lv->nblocks > 0)
        for (int l = 0; l < lv->level; l++)
            if (!lv->child[l]) return false;
    return true;
}

bool check_mesh(const geo_mesh* m) {
    if (!m) return false;
    if (m->nv < 0 || m->nt < 0) return false;
    if (m->vdtype != GEO_F32 && m->vdtype != GEO_F64) return false;
    if (m->nt > 0 && (!m->tris || !m->verts || m->nv == 0)) return false;
    if ((int64_t)m->nt * 3 > INT32_MAX || (int64_t)m->nv * 3 > INT32_MAX) return false;
    return true;
}

bool check_bins(const geo_bins* b, int kind, int64_t nkeys) {
    if (!b || b->kind != kind || b->nkeys != nkeys || !b->off || !b->d_count || b->cap < 0) return false;
    if (b->cap > 0 && !b->val) return false;
    if (b->cap > INT32_MAX) return false;
    return true;
}

int64_t row_keys(const geo_level* lv) {
    return ((int64_t)lv->n0[1] << lv->level) * ((int64_t)lv->n0[2] << lv->level);
}

}  // namespace

extern "C" {

size_t geo_workspace_size(int32_t call, int64_t nkeys, int64_t cap) {
    if (nkeys < 0) return 0;
    switch (call) {
        case GEO_CALL_BINS_ROWS:
        case GEO_CALL_BINS_LINKS: return bins_ws_bytes(nkeys, cap);
        case GEO_CALL_BINS_ROWS_LEVELS: return rows_levels_ws_bytes(nkeys, cap);
        case GEO_CALL_REFINE: return geo_refine_ws_bytes(nkeys);
        case GEO_CALL_CUTLINKS: return geo_cutlinks_ws_bytes(nkeys, cap);
        case GEO_CALL_LINKS_DENSE: return geo_dense_ws_bytes(nkeys);
        case GEO_CALL2_BINS: return geo2_bins_ws_bytes(nkeys);
        case GEO_CALL2_REFINE: return geo2_refine_ws_bytes(nkeys);
        case GEO_CALL2_CUTLINKS: return geo2_cutlinks_ws_bytes(nkeys);
        default: return 0;
    }
}

int32_t geo_nprop(double d_spec) {
    // N_prop - 1 = largest k >= 0 with k 4 sqrt(2) <= d_spec, i.e. 32 k^2 <= d_spec^2
    if (!(d_spec > 0) || !isfinite(d_spec)) return 1;
    int64_t k = (int64_t)floor(d_spec / (4.0 * sqrt(2.0)));
    if (k < 0) k = 0;
    // exact comparison of 32 k^2 with d^2 = p + e (p = d*d, e = fma(d, d, -p))
    auto le = [&](int64_t kk) {
        const double lhs = 32.0 * (double)kk * (double)kk;  // exact for kk < 2^24
        const double p = d_spec * d_spec, e = fma(d_spec, d_spec, -p);
        return lhs < p || (lhs == p && e >= 0);
    };
    while (k > 0 && !le(k)) k--;
    while (le(k + 1)) k++;
    return (int32_t)(1 + k);
}

int geo_level0_blocks(const int32_t n0[3], int32_t* bcoord, geo_stream_t stream) {
    if (!n0 || !bcoord) return GEO_ERR_ARG;
    for (int a = 0; a < 3; a++)
        if (n0[a] <= 0 || n0[a] % 4 != 0 || n0[a] > GEO_MAX_RES) return GEO_ERR_ARG;
    return launch_level0(n0, bcoord, (hipStream_t)stream);
}

int geo_build_bins(const geo_mesh* mesh, const geo_level* lv, int32_t kind, int32_t precision, geo_bins* out,
                   uint64_t* d_stats, void* ws, size_t ws_bytes, geo_stream_t stream) {
    if (!check_mesh(mesh) || !check_level(lv)) return GEO_ERR_ARG;
    if (kind != GEO_BINS_ROWS && kind != GEO_BINS_LINKS) return GEO_ERR_ARG;
    if (precision != GEO_PREC_F64 && precision != GEO_PREC_F32_FALLBACK) return GEO_ERR_ARG;
    const int64_t nkeys = kind == GEO_BINS_ROWS ? row_keys(lv) : (int64_t)lv->nblocks;
    if (!check_bins(out, kind, nkeys)) return GEO_ERR_ARG;
    if (nkeys + 1 > INT32_MAX) return GEO_ERR_ARG;
    if (ws_bytes < bins_ws_bytes(nkeys, out->cap) || (!ws && ws_bytes)) return GEO_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char* p = static_cast<char*>(ws);
    int2* pairs = reinterpret_cast<int2*>(p);
    p += al(sizeof(int2) * (size_t)out->cap);
    int32_t* rank = reinterpret_cast<int32_t*>(p);
    p += al(sizeof(int32_t) * (size_t)out->cap);
    int32_t* cnt = reinterpret_cast<int32_t*>(p);
    p += al(sizeof(int32_t) * ((size_t)nkeys + 1));
    int32_t* partials = reinterpret_cast<int32_t*>(p);
    const DevMesh m = dev_mesh(mesh);
    const DevLevel d = dev_level(lv);
    int rc;
    if ((rc = geo_zero_counts(reinterpret_cast<uint64_t*>(out->d_count), cnt, nkeys, s)) != GEO_OK) return rc;
    if ((rc = launch_check_mesh(m, d, d_stats, s)) != GEO_OK) return rc;
    if (kind == GEO_BINS_ROWS)
        rc = launch_rows_pass1(m, d, precision, cnt, pairs, rank, out->cap, out->d_count, d_stats, s);
    else
        rc = launch_links_pass1(m, d, cnt, pairs, rank, out->cap, out->d_count, s);
    if (rc != GEO_OK) return rc;
    if ((rc = geo_scan_exclusive(cnt, out->off, nkeys, partials, s)) != GEO_OK) return rc;
    return launch_bins_scatter(pairs, rank, out->cap, out->d_count, out->off, out->val, s);
}

int geo_build_row_bins_levels(const geo_mesh* mesh, const int32_t n0[3], int32_t lmin, int32_t nlev,
                              int32_t precision, const geo_bins* out, uint64_t* d_stats, void* ws, size_t ws_bytes,
                              geo_stream_t stream) {
    if (!check_mesh(mesh) || !n0 || !out) return GEO_ERR_ARG;
    if (lmin < 0 || nlev < 1 || lmin + nlev > GEO_MAX_LEVELS) return GEO_ERR_ARG;
    if (precision != GEO_PREC_F64 && precision != GEO_PREC_F32_FALLBACK) return GEO_ERR_ARG;
    geo_level lv{};
    for (int a = 0; a < 3; a++) lv.n0[a] = n0[a];
    lv.level = lmin + nlev - 1;  // the finest level bounds the resolution
    if (!check_level(&lv)) return GEO_ERR_ARG;
    RowLevels rl{};
    rl.nlev = nlev;
    rl.lmin = lmin;
    int64_t nkeys = 0, cap = 0;
    for (int l = 0; l < nlev; l++) {
        lv.level = lmin + l;
        const int64_t nk = row_keys(&lv);
        if (!check_bins(&out[l], GEO_BINS_ROWS, nk)) return GEO_ERR_ARG;
        for (int q = 0; q < l; q++)
            if (out[q].d_count == out[l].d_count) return GEO_ERR_ARG;  // each level counts on its own
        rl.base[l] = (int)nkeys;
        nkeys += nk;
        if (nkeys + 1 > INT32_MAX) return GEO_ERR_ARG;
        rl.count[l] = reinterpret_cast<unsigned long long*>(out[l].d_count);
        rl.off[l] = out[l].off;
        rl.val[l] = out[l].val;
        rl.cap[l] = out[l].cap;
        cap += out[l].cap;
    }
    for (int l = nlev; l <= GEO_MAX_LEVELS; l++) rl.base[l] = (int)nkeys;
    if (ws_bytes < rows_levels_ws_bytes(nkeys, cap) || (!ws && ws_bytes)) return GEO_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char* p = static_cast<char*>(ws);
    int2* pairs = reinterpret_cast<int2*>(p);
    p += al(sizeof(int2) * (size_t)cap);
    int32_t* rank = reinterpret_cast<int32_t*>(p);
    p += al(sizeof(int32_t) * (size_t)cap);
    int32_t* cnt = reinterpret_cast<int32_t*>(p);
    p += al(sizeof(int32_t) * ((size_t)nkeys + 1));
    int32_t* partials = reinterpret_cast<int32_t*>(p);
    p += al(geo_scan_partials_bytes(nkeys));
    int64_t* d_pairs = reinterpret_cast<int64_t*>(p);
    lv.level = lmin;
    const DevMesh m = dev_mesh(mesh);
    const DevLevel d = dev_level(&lv);
    int rc;
    if ((rc = launch_rows_levels_zero(rl, d_pairs, cnt, nkeys, s)) != GEO_OK) return rc;
    if ((rc = launch_check_mesh(m, d, d_stats, s)) != GEO_OK) return rc;
    if ((rc = launch_rows_levels(m, d, precision, rl, cnt, pairs, rank, cap, d_pairs, d_stats, s)) != GEO_OK)
        return rc;
    for (int l = 0; l < nlev; l++)
        if ((rc = geo_scan_exclusive(cnt + rl.base[l], out[l].off, out[l].nkeys, partials, s)) != GEO_OK) return rc;
    return launch_rows_levels_scatter(pairs, rank, cap, d_pairs, rl, s);
}

int geo_voxelize(const geo_level* lv, const geo_bins* rows, uint64_t* solid, geo_stream_t stream) {
    if (!check_level(lv) || !check_bins(rows, GEO_BINS_ROWS, row_keys(lv))) return GEO_ERR_ARG;
    if (lv->nblocks > 0 && !solid) return GEO_ERR_ARG;
    return launch_voxelize(dev_level(lv), rows->off, rows->val, rows->cap, solid, (hipStream_t)stream);
}

int geo_refine_flags(const geo_level* lv, const uint64_t* solid, int32_t n_prop, uint8_t* bclass, uint8_t* refine,
                     int32_t* child_map, int32_t* child_bcoord, int64_t* d_nchild, void* ws, size_t ws_bytes,
                     geo_stream_t stream) {
    if (!check_level(lv) || n_prop < 0 || !d_nchild) return GEO_ERR_ARG;
    if (lv->level + 1 >= GEO_MAX_LEVELS) return GEO_ERR_ARG;
    for (int a = 0; a < 3; a++)
        if ((int64_t)lv->n0[a] << (lv->level + 1) > GEO_MAX_RES) return GEO_ERR_ARG;
    if ((int64_t)lv->nblocks * 8 > INT32_MAX / 64) return GEO_ERR_ARG;
    if (lv->nblocks > 0 && (!solid || !bclass || !refine || !child_map || !child_bcoord)) return GEO_ERR_ARG;
    if (ws_bytes < geo_refine_ws_bytes(lv->nblocks) || (!ws && ws_bytes)) return GEO_ERR_WORKSPACE;
    return launch_refine(dev_level(lv), solid, n_prop, bclass, refine, child_map, child_bcoord, d_nchild, ws, ws_bytes,
                         (hipStream_t)stream);
}

int geo_cutlinks(const geo_mesh* mesh, const geo_level* lv, const geo_bins* rows, const geo_bins* links,
                 int32_t lattice, int32_t precision, uint32_t* link_mask, int64_t cap, int64_t* d_nlinks,
                 int32_t* link_cell, uint8_t* link_dir, float* link_q, int32_t* link_tri, uint64_t* d_stats,
                 void* ws, size_t ws_bytes, geo_stream_t stream) {
    if (!check_mesh(mesh) || !check_level(lv)) return GEO_ERR_ARG;
    if (!check_bins(rows, GEO_BINS_ROWS, row_keys(lv)) || !check_bins(links, GEO_BINS_LINKS, lv->nblocks))
        return GEO_ERR_ARG;
    if (lattice != 19 && lattice != 27) return GEO_ERR_ARG;
    if (precision != GEO_PREC_F64 && precision != GEO_PREC_F32_FALLBACK) return GEO_ERR_ARG;
    if (cap < 0 || !d_nlinks) return GEO_ERR_ARG;
    if (cap > 0 && (!link_cell || !link_dir || !link_q || !link_tri)) return GEO_ERR_ARG;
    if (mesh->nt >= (1 << 27)) return GEO_ERR_ARG;  // hit keys hold 27-bit triangle ids
    if (ws_bytes < geo_cutlinks_ws_bytes(lv->nblocks, cap) || (!ws && ws_bytes)) return GEO_ERR_WORKSPACE;
    return launch_cutlinks(dev_mesh(mesh), dev_level(lv), rows, links, lattice, precision, link_mask, cap, d_nlinks,
                           link_cell, link_dir, link_q, link_tri, d_stats, ws, ws_bytes, (hipStream_t)stream);
}

int geo_cutlinks_backward(const geo_mesh* mesh, const geo_level* lv, int64_t n_links, const int32_t* link_cell,
                          const uint8_t* link_dir, const int32_t* link_tri, const float* grad_q, float* grad_verts,
                          geo_stream_t stream) {
    if (!check_mesh(mesh) || !check_level(lv) || n_links < 0) return GEO_ERR_ARG;
    if (n_links > 0 && (!link_cell || !link_dir || !link_tri || !grad_q || !grad_verts)) return GEO_ERR_ARG;
    return launch_backward(dev_mesh(mesh), dev_level(lv), n_links, link_cell, link_dir, link_tri, grad_q, grad_verts,
                           (hipStream_t)stream);
}

int geo_links_dense(const geo_level* lv, int64_t n_links, const int32_t* link_cell, const uint8_t* link_dir,
                    const float* link_q, const int32_t* link_tri, int32_t lattice, int64_t cap, int32_t* block_map,
                    float* dense_q, int32_t* dense_tri, int64_t* d_nbnd, void* ws, size_t ws_bytes,
                    geo_stream_t stream) {
    if (!check_level(lv) || n_links < 0 || cap < 0 || !d_nbnd) return GEO_ERR_ARG;
    if (lattice != 19 && lattice != 27) return GEO_ERR_ARG;
    if (n_links > 0 && (!link_cell || !link_dir || !link_q || !link_tri)) return GEO_ERR_ARG;
    if (lv->nblocks > 0 && !block_map) return GEO_ERR_ARG;
    if (cap > 0 && (!dense_q || !dense_tri)) return GEO_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(dense_q) | reinterpret_cast<uintptr_t>(dense_tri)) & 15) return GEO_ERR_ARG;
    if (!ws && ws_bytes) return GEO_ERR_WORKSPACE;
    return launch_links_dense(lv->nblocks, n_links, link_cell, link_dir, link_q, link_tri, lattice, cap, block_map,
                              dense_q, dense_tri, d_nbnd, ws, ws_bytes, (hipStream_t)stream);
}

int geo_block_neighbours(const geo_level* lv, int32_t* nbr, geo_stream_t stream) {
    if (!check_level(lv)) return GEO_ERR_ARG;
    if (lv->nblocks > 0 && !nbr) return GEO_ERR_ARG;
    return launch_block_nbr(dev_level(lv), nbr, (hipStream_t)stream);
}

int geo_ibb(const geo_level* lv, const uint64_t* solid, const int32_t* block_map, const float* dense_q,
            int64_t nbnd, const int32_t* nbr, int32_t lattice, int32_t interpolate, int32_t dtype,
            const void* f_post, void* f_new, uint64_t* d_fallback, geo_stream_t stream) {
    if (!check_level(lv) || nbnd < 0) return GEO_ERR_ARG;
    if ((lattice != 19 && lattice != 27) || (dtype != GEO_F32 && dtype != GEO_F64)) return GEO_ERR_ARG;
    if (lv->nblocks > 0 && (!solid || !block_map || !f_post || !f_new)) return GEO_ERR_ARG;
    if (nbnd > 0 && !dense_q) return GEO_ERR_ARG;
    if (lv->nblocks > 0) {
        // the two population arrays must not overlap
        const size_t bytes =
            (size_t)lv->nblocks * (lattice == 27 ? 27 : 19) * 64 * (dtype == GEO_F64 ? sizeof(double) : sizeof(float));
        const uintptr_t a = reinterpret_cast<uintptr_t>(f_post), b = reinterpret_cast<uintptr_t>(f_new);
        if (a < b + bytes && b < a + bytes) return GEO_ERR_ARG;
    }
    return launch_ibb(dev_level(lv), solid, block_map, dense_q, nbnd, nbr, lattice, interpolate, dtype, f_post, f_new,
                      reinterpret_cast<unsigned long long*>(d_fallback), (hipStream_t)stream);
}

int geo_solid_change(int64_t nblocks, const uint64_t* prev, const uint64_t* cur, uint64_t* spawned,
                     uint64_t* covered, int64_t* d_counts, geo_stream_t stream) {
    if (nblocks < 0 || !d_counts) return GEO_ERR_ARG;
    if (nblocks > 0 && (!prev || !cur)) return GEO_ERR_ARG;
    return launch_solid_change(nblocks, prev, cur, spawned, covered, reinterpret_cast<unsigned long long*>(d_counts),
                               (hipStream_t)stream);
}

const char* geo_version(void) { return "libgeo 0.2 (gfx950)"; }

}  // extern "C"
