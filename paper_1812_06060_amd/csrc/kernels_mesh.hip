// Mesh geometry on the GPU (Sec. 3.1): face areas, corner cotangents,
// cotangent weights theta_jk = (cot a + cot b)/2, lumped vertex areas
// A_j = (1/3) sum of incident face areas, mean edge length (Eq. 27), unit
// edge vectors; plus caller<->internal permutations and the deterministic
// two-stage reductions used by convergence checks.
#include <cmath>

#include "hgeo_internal.h"

namespace hg {

constexpr int kBlock = 256;

// ---------------------------------------------------------------- reductions
// Block-wide sum / max of one double per thread; result valid in thread 0.
__device__ inline double block_reduce(double v, bool is_max) {
    __shared__ double sh[kBlock / 64];
    for (int o = 32; o > 0; o >>= 1) {
        double other = __shfl_down(v, o, 64);
        v = is_max ? fmax(v, other) : v + other;
    }
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = sh[0];
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = is_max ? fmax(r, sh[i]) : r + sh[i];
        v = r;
    }
    __syncthreads();
    return v;
}

__global__ void k_reduce_final(double* partial, int n, int is_max) {
    double acc = is_max ? -INFINITY : 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc = is_max ? fmax(acc, partial[i]) : acc + partial[i];
    acc = block_reduce(acc, is_max);
    if (threadIdx.x == 0) partial[n] = acc;
}

double reduce_partials(Mesh& m, Work& w, int nblocks, bool is_max, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, s, w.partial.p, nblocks, is_max ? 1 : 0);
    HG_CHECK_HIP(hipGetLastError());
    HG_CHECK_HIP(hipMemcpyAsync(w.pinned, w.partial.p + nblocks, sizeof(double), hipMemcpyDeviceToHost, s));
    HG_CHECK_HIP(hipStreamSynchronize(s));
    (void)m;
    return *w.pinned;
}

// ------------------------------------------------------------------ geometry
__device__ inline void load3(const double* x, const double* y, const double* z, int i, double p[3]) {
    p[0] = x[i];
    p[1] = y[i];
    p[2] = z[i];
}
__device__ inline void sub3(const double a[3], const double b[3], double r[3]) {
    r[0] = a[0] - b[0];
    r[1] = a[1] - b[1];
    r[2] = a[2] - b[2];
}
__device__ inline void cross3(const double a[3], const double b[3], double r[3]) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ inline double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Corner positions of face f: from the vertex positions, or (intrinsic
// meshes, floc != null) the face's own plane: (0,0,0), (l01,0,0), (x2,y2,0).
__device__ inline void face_corners(int f, const int32_t* tri, const double* px, const double* py, const double* pz,
                                    const double* floc, double p[3][3]) {
    if (floc) {
        p[0][0] = p[0][1] = p[0][2] = 0.0;
        p[1][0] = floc[3 * f];
        p[1][1] = p[1][2] = 0.0;
        p[2][0] = floc[3 * f + 1];
        p[2][1] = floc[3 * f + 2];
        p[2][2] = 0.0;
    } else {
        for (int k = 0; k < 3; ++k) load3(px, py, pz, tri[3 * f + k], p[k]);
    }
}

// Per face: area and the cotangent of each corner angle; flags degenerate faces.
__global__ void k_face_geom(int nf, const int32_t* tri, const double* px, const double* py, const double* pz,
                            const double* floc, double* farea, double* fcot, int* bad, double* partial) {
    int f = blockIdx.x * blockDim.x + threadIdx.x;
    double a2 = 0.0;
    if (f < nf) {
        double p[3][3];
        face_corners(f, tri, px, py, pz, floc, p);
        double e1[3], e2[3], n[3];
        sub3(p[1], p[0], e1);
        sub3(p[2], p[0], e2);
        cross3(e1, e2, n);
        double dbl = sqrt(dot3(n, n));
        farea[f] = 0.5 * dbl;
        a2 = 0.5 * dbl;
        if (!(dbl > 0.0)) bad[0] = 1;
        for (int k = 0; k < 3; ++k) {
            double u[3], w[3];
            sub3(p[(k + 1) % 3], p[k], u);
            sub3(p[(k + 2) % 3], p[k], w);
            fcot[3 * f + k] = dot3(u, w) / dbl;
        }
    }
    double s = block_reduce(a2, false);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Per edge: theta_e = sum over incident faces of cot(opposite corner)/2, and
// the edge length (partial sums for the mean).
__global__ void k_edge_theta(int ne, const int32_t* ev, const int32_t* ef, const uint32_t* fslot,
                             const double* fcot, const double* px, const double* py, const double* pz,
                             const double* elen, double* theta_e, double* partial) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    double len = 0.0;
    if (e < ne) {
        double th = 0.0;
        for (int s = 0; s < 2; ++s) {
            int f = ef[2 * e + s];
            if (f < 0) continue;
            for (int k = 0; k < 3; ++k)
                if (slot_edge(fslot[3 * f + k]) == e) th += 0.5 * fcot[3 * f + (k + 2) % 3];
        }
        theta_e[e] = th;
        if (elen) {   // intrinsic: the lengths of the flipped triangulation
            len = elen[e];
        } else {
            double a[3], b[3], d[3];
            load3(px, py, pz, ev[2 * e], a);
            load3(px, py, pz, ev[2 * e + 1], b);
            sub3(b, a, d);
            len = sqrt(dot3(d, d));
        }
    }
    double s = block_reduce(len, false);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Per vertex: CSR weights, their row sum, and the lumped area.  Each face at
// v_j is reached through its two edges at v_j, hence the factor 1/6.
__global__ void k_vertex_fill(int nv, const int32_t* row_ptr, const int32_t* csr_edge, const int32_t* ef,
                              const double* theta_e, const double* farea, double* theta, double* sum_theta,
                              double* Av) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nv) return;
    double st = 0.0, ar = 0.0;
    for (int k = row_ptr[j]; k < row_ptr[j + 1]; ++k) {
        int e = csr_edge[k];
        double th = theta_e[e];
        theta[k] = th;
        st += th;
        for (int s = 0; s < 2; ++s) {
            int f = ef[2 * e + s];
            if (f >= 0) ar += farea[f];
        }
    }
    sum_theta[j] = st;
    Av[j] = ar / 6.0;
}

// Per face slot (face form): the unit vector of the slot's edge (along its
// orientation halfedge) and the weight A_nb / (A_own + A_nb) of the
// neighbour across it (0 on the boundary).
__global__ void k_slot_geom(int nf, const uint32_t* fslot, const int32_t* twin, const int32_t* ev, const double* px,
                            const double* py, const double* pz, const double* farea, float4* sgeo) {
    int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= 3 * nf) return;
    const int e = slot_edge(fslot[h]);
    double a[3], b[3], d[3];
    load3(px, py, pz, ev[2 * e], a);
    load3(px, py, pz, ev[2 * e + 1], b);
    sub3(b, a, d);
    const double len = sqrt(dot3(d, d));
    const int t = twin[h];
    float w = 0.f;
    if (t >= 0) {
        const float Af = (float)farea[h / 3], An = (float)farea[t / 3];
        w = An / (Af + An);
    }
    sgeo[h] = make_float4((float)(d[0] / len), (float)(d[1] / len), (float)(d[2] / len), w);
}

void Mesh::ensure_sgeo(hipStream_t s) {
    std::lock_guard<std::mutex> lock(sgeo_mu);
    if (sgeo.p) return;
    DBuf<float4> tmp;
    tmp.alloc((size_t)3 * nf);
    hipLaunchKernelGGL(k_slot_geom, dim3(grid_for(3 * nf, kBlock)), dim3(kBlock), 0, s, (int)nf, fslot.p, twin.p,
                       ev.p, px.p, py.p, pz.p, farea.p, tmp.p);
    HG_CHECK_HIP(hipGetLastError());
    HG_CHECK_HIP(hipStreamSynchronize(s));   // other queries may read it as soon as the lock is released
    std::swap(sgeo.p, tmp.p);
    std::swap(sgeo.n, tmp.n);
}

void geometry_init(Mesh& m, hipStream_t s, const std::vector<double>* elen_host) {
    const int nf = (int)m.nf, ne = (int)m.ne, nv = (int)m.nv;
    DBuf<double> fcot, theta_e, elen;
    if (elen_host) elen.upload(*elen_host, s);
    DBuf<int> bad;
    fcot.alloc((size_t)3 * nf);
    theta_e.alloc(ne);
    bad.alloc(1);
    HG_CHECK_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
    m.farea.alloc(nf);
    m.theta.alloc((size_t)2 * ne);
    m.sum_theta.alloc(nv);
    m.Av.alloc(nv);
    int gf = grid_for(nf, kBlock), ge = grid_for(ne, kBlock);
    m.w.partial.alloc((size_t)std::max(gf, ge) + 8);
    hipLaunchKernelGGL(k_face_geom, dim3(gf), dim3(kBlock), 0, s, nf, m.tri.p, m.px.p, m.py.p, m.pz.p,
                       m.intrinsic ? m.floc.p : nullptr, m.farea.p, fcot.p, bad.p, m.w.partial.p);
    HG_CHECK_HIP(hipGetLastError());
    m.total_area = reduce_partials(m, m.w, gf, false, s);
    int hbad = 0;
    HG_CHECK_HIP(hipMemcpy(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost));
    if (hbad) throw Error{HG_E_BAD_MESH, "zero-area face"};
    hipLaunchKernelGGL(k_edge_theta, dim3(ge), dim3(kBlock), 0, s, ne, m.ev.p, m.ef.p, m.fslot.p, fcot.p, m.px.p,
                       m.py.p, m.pz.p, elen_host ? elen.p : nullptr, theta_e.p, m.w.partial.p);
    HG_CHECK_HIP(hipGetLastError());
    const double hb = reduce_partials(m, m.w, ge, false, s) / (double)ne;
    if (!m.intrinsic) m.hbar = hb;   // intrinsic: the input mesh's mean edge length, set by the caller
    hipLaunchKernelGGL(k_vertex_fill, dim3(grid_for(nv, kBlock)), dim3(kBlock), 0, s, nv, m.row_ptr.p,
                       m.csr_edge.p, m.ef.p, theta_e.p, m.farea.p, m.theta.p, m.sum_theta.p, m.Av.p);
    HG_CHECK_HIP(hipGetLastError());
    HG_CHECK_HIP(hipStreamSynchronize(s));
}

// -------------------------------------------------------------- permutations
template <class T>
__global__ void k_scatter(int n, const int32_t* perm, const T* in, T* out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[perm[i]] = in[i];
}
template <class T>
__global__ void k_gather(int n, const int32_t* perm, const T* in, T* out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[perm[i]];
}
__global__ void k_scatter3(int n, const int32_t* perm, const float* in, float* out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        int u = perm[i];
        out[3 * u] = in[3 * i];
        out[3 * u + 1] = in[3 * i + 1];
        out[3 * u + 2] = in[3 * i + 2];
    }
}
__global__ void k_gather3(int n, const int32_t* perm, const float* in, float* out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        int u = perm[i];
        out[3 * i] = in[3 * u];
        out[3 * i + 1] = in[3 * u + 1];
        out[3 * i + 2] = in[3 * u + 2];
    }
}
// Internal int values (vertex ids or -1) to caller order, optionally mapping
// the values themselves through perm_v.
__global__ void k_scatter_ids(int n, const int32_t* perm, const int32_t* in, int32_t* out, int map_values) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        int v = in[i];
        if (map_values && v >= 0) v = perm[v];
        out[perm[i]] = v;
    }
}
__global__ void k_edges_user(int ne, const int32_t* perm_e, const int32_t* perm_v, const int32_t* ev, int32_t* out) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < ne) {
        int a = perm_v[ev[2 * e]], b = perm_v[ev[2 * e + 1]];
        int r = perm_e[e];
        out[2 * r] = a < b ? a : b;
        out[2 * r + 1] = a < b ? b : a;
    }
}

void scatter_faces_to_user(Mesh& m, const float* in, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter3, dim3(grid_for(m.nf, kBlock)), dim3(kBlock), 0, s, (int)m.nf, m.perm_f.p, in, out);
    HG_CHECK_HIP(hipGetLastError());
}
void gather_faces_to_internal(Mesh& m, const float* in, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_gather3, dim3(grid_for(m.nf, kBlock)), dim3(kBlock), 0, s, (int)m.nf, m.perm_f.p, in, out);
    HG_CHECK_HIP(hipGetLastError());
}
void scatter_edges_to_user(Mesh& m, const float* in, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter<float>, dim3(grid_for(m.ne, kBlock)), dim3(kBlock), 0, s, (int)m.ne, m.perm_e.p, in,
                       out);
    HG_CHECK_HIP(hipGetLastError());
}
void gather_edges_to_internal(Mesh& m, const float* in, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_gather<float>, dim3(grid_for(m.ne, kBlock)), dim3(kBlock), 0, s, (int)m.ne, m.perm_e.p, in,
                       out);
    HG_CHECK_HIP(hipGetLastError());
}
void scatter_vertices_to_user_d(Mesh& m, const double* in, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter<double>, dim3(grid_for(m.nv, kBlock)), dim3(kBlock), 0, s, (int)m.nv, m.perm_v.p,
                       in, out);
    HG_CHECK_HIP(hipGetLastError());
}
void gather_vertices_to_internal_d(Mesh& m, const double* in, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_gather<double>, dim3(grid_for(m.nv, kBlock)), dim3(kBlock), 0, s, (int)m.nv, m.perm_v.p,
                       in, out);
    HG_CHECK_HIP(hipGetLastError());
}
void scatter_vertices_to_user_i(Mesh& m, const int32_t* in, int32_t* out, bool map_values, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_ids, dim3(grid_for(m.nv, kBlock)), dim3(kBlock), 0, s, (int)m.nv, m.perm_v.p, in,
                       out, map_values ? 1 : 0);
    HG_CHECK_HIP(hipGetLastError());
}
// theta of each edge from its CSR entry at the smaller internal endpoint,
// into the canonical edge order
__global__ void k_theta_user(int nv, const int32_t* row_ptr, const int32_t* col, const int32_t* csr_edge,
                             const double* theta, const int32_t* perm_e, double* out) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nv) return;
    for (int k = row_ptr[j]; k < row_ptr[j + 1]; ++k)
        if (col[k] > j) out[perm_e[csr_edge[k]]] = theta[k];
}

void weights_to_user(Mesh& m, double* theta_user, double* area_user, hipStream_t s) {
    if (theta_user) {
        hipLaunchKernelGGL(k_theta_user, dim3(grid_for(m.nv, kBlock)), dim3(kBlock), 0, s, (int)m.nv, m.row_ptr.p,
                           m.col.p, m.csr_edge.p, m.theta.p, m.perm_e.p, theta_user);
        HG_CHECK_HIP(hipGetLastError());
    }
    if (area_user) scatter_vertices_to_user_d(m, m.Av.p, area_user, s);
}

void edges_to_user(Mesh& m, int32_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_edges_user, dim3(grid_for(m.ne, kBlock)), dim3(kBlock), 0, s, (int)m.ne, m.perm_e.p,
                       m.perm_v.p, m.ev.p, out);
    HG_CHECK_HIP(hipGetLastError());
}

}  // namespace hg
