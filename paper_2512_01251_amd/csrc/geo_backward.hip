// Backward of the cut-link lengths q with respect to the mesh vertices.
//
// q = n.(a - x) / (n.d) for the hit triangle (a, b, c), n = (b-a) x (c-a),
// d = h c_k.  Moving vertex v_j by dv moves the surface at the hit point by
// lambda_j dv (barycentric coordinate of the hit point), and the hit slides
// along d until n.(dq d) = n.(lambda_j dv), so dq/dv_j = lambda_j n / (n.d).
// One thread per link; float64 arithmetic, float32 atomic accumulation.
#include "geo_internal.h"

namespace {

__global__ void k_backward(DevMesh m, DevLevel d, int64_t n_links, const int32_t* link_cell, const uint8_t* link_dir,
                           const int32_t* link_tri, const float* grad_q, float* grad) {
    const double h = ldexp(1.0, -d.level);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_links; i += (int64_t)gridDim.x * blockDim.x) {
        const int tri = link_tri[i];
        const float g = grad_q[i];
        if (tri < 0 || tri >= m.nt || g == 0.0f) continue;
        const int cell = link_cell[i];
        const int64_t b = cell >> 6;
        if (b >= d.nblocks) continue;
        const int t = cell & 63;
        const int k = link_dir[i];
        const double X[3] = {(4 * d.bcoord[3 * b] + (t & 3) + 0.5) * h, (4 * d.bcoord[3 * b + 1] + ((t >> 2) & 3) + 0.5) * h,
                             (4 * d.bcoord[3 * b + 2] + (t >> 4) + 0.5) * h};
        const double dv[3] = {(k % 3 - 1) * h, ((k / 3) % 3 - 1) * h, (k / 9 - 1) * h};
        int vid[3];
        double P[3][3];
        for (int j = 0; j < 3; j++) {
            vid[j] = m.tris[3 * (int64_t)tri + j];
            for (int a = 0; a < 3; a++) P[j][a] = load_coord(m, vid[j], a);
        }
        const double e1[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
        const double e2[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
        const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        const double nd = n[0] * dv[0] + n[1] * dv[1] + n[2] * dv[2];
        const double nn = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
        if (nd == 0.0 || nn == 0.0) continue;
        const double q = (n[0] * (P[0][0] - X[0]) + n[1] * (P[0][1] - X[1]) + n[2] * (P[0][2] - X[2])) / nd;
        const double H[3] = {X[0] + q * dv[0], X[1] + q * dv[1], X[2] + q * dv[2]};
        for (int j = 0; j < 3; j++) {
            const double* u = P[(j + 1) % 3];
            const double* w = P[(j + 2) % 3];
            const double uu[3] = {u[0] - H[0], u[1] - H[1], u[2] - H[2]};
            const double ww[3] = {w[0] - H[0], w[1] - H[1], w[2] - H[2]};
            const double cr[3] = {uu[1] * ww[2] - uu[2] * ww[1], uu[2] * ww[0] - uu[0] * ww[2], uu[0] * ww[1] - uu[1] * ww[0]};
            const double lam = (n[0] * cr[0] + n[1] * cr[1] + n[2] * cr[2]) / nn;
            const double f = (double)g * lam / nd;
            for (int a = 0; a < 3; a++) unsafeAtomicAdd(&grad[3 * (int64_t)vid[j] + a], (float)(f * n[a]));
        }
    }
}

}  // namespace

int launch_backward(const DevMesh& m, const DevLevel& d, int64_t n_links, const int32_t* link_cell,
                    const uint8_t* link_dir, const int32_t* link_tri, const float* grad_q, float* grad_verts,
                    hipStream_t s) {
    if (n_links <= 0) return GEO_OK;
    int64_t g = (n_links + 255) / 256;
    if (g > 65536) g = 65536;
    k_backward<<<(unsigned)g, 256, 0, s>>>(m, d, n_links, link_cell, link_dir, link_tri, grad_q, grad_verts);
    GEO_LAUNCH_CHECK();
    return GEO_OK;
}
