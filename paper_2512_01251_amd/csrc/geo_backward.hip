// Backward of the cut-link lengths q with respect to the mesh vertices.
//
// q = n.(a - x) / (n.d) for the hit triangle (a, b, c), n = (b-a) x (c-a),
// d = h c_k.  Moving vertex v_j by dv moves the surface at the hit point by
// lambda_j dv (barycentric coordinate of the hit point), and the hit slides
// along d until n.(dq d) = n.(lambda_j dv), so dq/dv_j = lambda_j n / (n.d).
// One thread per link; float64 arithmetic.  Contributions are summed per
// vertex before they reach HBM: runs of one vertex among consecutive lanes by
// segmented prefix sums, then per round of 256 links in an LDS table (links
// next to each other in the table come from neighbouring cells and hit the
// same few triangles); each distinct vertex of a round takes one float32
// atomic add per component in HBM.
#include "geo_internal.h"

namespace {

constexpr int BW_THREADS = 256;
constexpr int BW_SLOTS = 1024;  // > 3 * BW_THREADS: a round never fills the table

__device__ __forceinline__ unsigned bw_hash(int v) { return ((unsigned)v * 2654435761u) >> 22; }


__global__ void __launch_bounds__(BW_THREADS) k_backward(DevMesh m, DevLevel d, int64_t n_links,
                                                         const int32_t* link_cell, const uint8_t* link_dir,
                                                         const int32_t* link_tri, const float* grad_q, float* grad) {
    __shared__ int skey[BW_SLOTS];
    __shared__ float sval[BW_SLOTS][3];
    for (int i = threadIdx.x; i < BW_SLOTS; i += BW_THREADS) {
        skey[i] = -1;
        sval[i][0] = sval[i][1] = sval[i][2] = 0.0f;
    }
    __syncthreads();
    const double h = ldexp(1.0, -d.level);
    const int64_t stride = (int64_t)gridDim.x * BW_THREADS;
    for (int64_t base = (int64_t)blockIdx.x * BW_THREADS; base < n_links; base += stride) {
        const int64_t i = base + threadIdx.x;
        int vid[3] = {-1, -1, -1};
        float contrib[3][3];
        if (i < n_links) {
            const int tri = link_tri[i];
            const float g = grad_q[i];
            const int cell = link_cell[i];
            const int64_t b = cell >> 6;
            if (tri >= 0 && tri < m.nt && g != 0.0f && b < d.nblocks) {
                const int t = cell & 63;
                const int k = link_dir[i];
                const double X[3] = {(4 * d.bcoord[3 * b] + (t & 3) + 0.5) * h,
                                     (4 * d.bcoord[3 * b + 1] + ((t >> 2) & 3) + 0.5) * h,
                                     (4 * d.bcoord[3 * b + 2] + (t >> 4) + 0.5) * h};
                const double dv[3] = {(k % 3 - 1) * h, ((k / 3) % 3 - 1) * h, (k / 9 - 1) * h};
                int vv[3];
                double P[3][3];
                for (int j = 0; j < 3; j++) {
                    vv[j] = m.tris[3 * (int64_t)tri + j];
                    for (int a = 0; a < 3; a++) P[j][a] = load_coord(m, vv[j], a);
                }
                const double e1[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
                const double e2[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
                const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                                     e1[0] * e2[1] - e1[1] * e2[0]};
                const double nd = n[0] * dv[0] + n[1] * dv[1] + n[2] * dv[2];
                const double nn = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
                if (nd != 0.0 && nn != 0.0) {
                    const double q = (n[0] * (P[0][0] - X[0]) + n[1] * (P[0][1] - X[1]) + n[2] * (P[0][2] - X[2])) / nd;
                    const double H[3] = {X[0] + q * dv[0], X[1] + q * dv[1], X[2] + q * dv[2]};
                    for (int j = 0; j < 3; j++) {
                        const double* u = P[(j + 1) % 3];
                        const double* w = P[(j + 2) % 3];
                        const double uu[3] = {u[0] - H[0], u[1] - H[1], u[2] - H[2]};
                        const double ww[3] = {w[0] - H[0], w[1] - H[1], w[2] - H[2]};
                        const double cr[3] = {uu[1] * ww[2] - uu[2] * ww[1], uu[2] * ww[0] - uu[0] * ww[2],
                                              uu[0] * ww[1] - uu[1] * ww[0]};
                        const double lam = (n[0] * cr[0] + n[1] * cr[1] + n[2] * cr[2]) / nn;
                        const double f = (double)g * lam / nd;
                        vid[j] = vv[j];
                        for (int a = 0; a < 3; a++) contrib[j][a] = (float)(f * n[a]);
                    }
                }
            }
        }
        // Neighbouring links of the table (one cell, successive directions)
        // often share a vertex: runs of equal vertex ids among consecutive
        // lanes are summed first (segmented prefix sums), and only the last
        // lane of a run adds into the LDS table (open addressing).
        const int lane = threadIdx.x & 63;
        for (int j = 0; j < 3; j++) {
            const int v = vid[j];
            float c0 = v >= 0 ? contrib[j][0] : 0.0f, c1 = v >= 0 ? contrib[j][1] : 0.0f,
                  c2 = v >= 0 ? contrib[j][2] : 0.0f;
            const int vprev = __shfl_up(v, 1, 64);
            int head = (lane == 0 || vprev != v) ? 1 : 0;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const float u0 = __shfl_up(c0, o, 64), u1 = __shfl_up(c1, o, 64), u2 = __shfl_up(c2, o, 64);
                const int hu = __shfl_up(head, o, 64);
                if (lane >= o) {
                    if (!head) {
                        c0 += u0;
                        c1 += u1;
                        c2 += u2;
                    }
                    head |= hu;
                }
            }
            const int vnext = __shfl_down(v, 1, 64);
            if (v < 0 || !(lane == 63 || vnext != v)) continue;
            unsigned slot = bw_hash(v);
            while (true) {
                const int prev = atomicCAS(&skey[slot], -1, v);
                if (prev == -1 || prev == v) break;
                slot = (slot + 1) & (BW_SLOTS - 1);
            }
            atomicAdd(&sval[slot][0], c0);
            atomicAdd(&sval[slot][1], c1);
            atomicAdd(&sval[slot][2], c2);
        }
        __syncthreads();
        // one global add per distinct vertex and component, then clear
        for (int sidx = threadIdx.x; sidx < BW_SLOTS; sidx += BW_THREADS) {
            const int v = skey[sidx];
            if (v >= 0) {
                for (int a = 0; a < 3; a++) unsafeAtomicAdd(&grad[3 * (int64_t)v + a], sval[sidx][a]);
                skey[sidx] = -1;
                sval[sidx][0] = sval[sidx][1] = sval[sidx][2] = 0.0f;
            }
        }
        __syncthreads();
    }
}

}  // namespace

int launch_backward(const DevMesh& m, const DevLevel& d, int64_t n_links, const int32_t* link_cell,
                    const uint8_t* link_dir, const int32_t* link_tri, const float* grad_q, float* grad_verts,
                    hipStream_t s) {
    if (n_links <= 0) return GEO_OK;
    int64_t g = (n_links + BW_THREADS - 1) / BW_THREADS;
    if (g > 16384) g = 16384;
    k_backward<<<(unsigned)g, BW_THREADS, 0, s>>>(m, d, n_links, link_cell, link_dir, link_tri, grad_q, grad_verts);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}
