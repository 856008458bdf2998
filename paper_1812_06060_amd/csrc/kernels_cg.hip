// Conjugate gradients for the heat method's two linear systems: the
// comparator of Sec. 6.4, where the direct solver of the original heat
// method is replaced by CG with a diagonal (Jacobi) preconditioner and the
// accuracy reached is set against computing time.
//
//   heat:    (A - t L_c) u = u_0 (Eq. 4), A lumped areas, u_0 = 1 at sources;
//   face:    K d = r, K = -L_c the cotangent stiffness, r_i = sum_f A_f
//            grad phi_i|_f . h_f (the Poisson step of Sec. 3.2);
//   edge:    L_E d = b_E, L_E the graph Laplacian with edge weight |H_e| (the
//            faces of the edge), b_E,i = sum_{f ni i} h_f . (2 p_i - p_j - p_k)
//            (the normal equations of Eqs. 19-20 on a closed field);
// the Poisson systems with d = 0 at every source, which the paper does to
// make the semi-definite system definite, and at vertices no source reaches.
//
// FP64 throughout, in the mesh's internal vertex order; the operator is
// applied row by row from the CSR one-ring (the cotangent weights theta of
// the mesh, or the face count of each edge).  Every reduction is two-level
// with a fixed partition and a fixed final order, so a run is
// deterministic; the CG scalars stay on the device (no host round trip per
// iteration).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "hgeo_internal.h"

namespace hg {

constexpr int kBlockC = 256;
constexpr int kCgCheck = 16;   // iterations between convergence checks

enum { CG_HEAT = 0, CG_FACE = 1, CG_EDGE = 2 };
// device scalars: rz of even / odd iterations, p.q, r.r, b.b
enum { S_RZ0 = 0, S_RZ1 = 1, S_PQ = 2, S_RR = 3, S_BB = 4, S_N = 8 };

struct CgOp {
    int op;
    const int32_t *row_ptr, *col, *csr_edge, *ef, *comp;
    const double *theta, *Av, *sum_theta, *tcomp;
};

__device__ inline double edge_weight(const CgOp& M, int k) {
    const int e = M.csr_edge[k];
    return (double)((M.ef[2 * e] >= 0) + (M.ef[2 * e + 1] >= 0));
}

// (operator x)_i, and its diagonal entry
__device__ inline double apply_row(const CgOp& M, int i, const double* __restrict__ x, double* diag) {
    const int k0 = M.row_ptr[i], k1 = M.row_ptr[i + 1];
    double off = 0.0, wsum = 0.0;
    for (int k = k0; k < k1; ++k) {
        const double w = M.op == CG_EDGE ? edge_weight(M, k) : M.theta[k];
        wsum += w;
        off = fma(w, x[M.col[k]], off);
    }
    double d;
    if (M.op == CG_HEAT) {
        const double t = M.tcomp[M.comp[i]];
        d = M.Av[i] + t * M.sum_theta[i];
        off *= t;
    } else {
        d = M.op == CG_FACE ? M.sum_theta[i] : wsum;
    }
    *diag = d;
    return d * x[i] - off;
}

template <int NV>
__device__ inline void block_sums(double (&v)[NV], double* __restrict__ partial, int stride) {
    __shared__ double sh[NV][kBlockC / 64];
#pragma unroll
    for (int j = 0; j < NV; ++j)
        for (int o = 32; o > 0; o >>= 1) v[j] += __shfl_down(v[j], o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < NV; ++j) sh[j][wid] = v[j];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            double s = 0.0;
            for (int q = 0; q < kBlockC / 64; ++q) s += sh[j][q];
            partial[j * stride + blockIdx.x] = s;
        }
}

// dst[dst_idx[j]] = sum over blocks of partial[j * stride + b], j < nvals
// (one workgroup; each thread sums a fixed strided subset, then a fixed tree)
__global__ void __launch_bounds__(kBlockC) k_cg_reduce(const double* __restrict__ partial, int nb, int stride,
                                                       int nvals, int d0, int d1, int d2, double* scal) {
    __shared__ double sh[kBlockC];
    const int dst[3] = {d0, d1, d2};
    for (int j = 0; j < nvals; ++j) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += kBlockC) s += partial[j * stride + b];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int h = kBlockC / 2; h > 0; h >>= 1) {
            if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) scal[dst[j]] = sh[0];
        __syncthreads();
    }
}

__global__ void k_cg_diag(int n, CgOp M, const uint8_t* __restrict__ fixed, double* __restrict__ D) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (fixed[i]) {
        D[i] = 1.0;
        return;
    }
    const int k0 = M.row_ptr[i], k1 = M.row_ptr[i + 1];
    double d;
    if (M.op == CG_HEAT) {
        d = M.Av[i] + M.tcomp[M.comp[i]] * M.sum_theta[i];
    } else if (M.op == CG_FACE) {
        d = M.sum_theta[i];
    } else {
        d = 0.0;
        for (int k = k0; k < k1; ++k) d += edge_weight(M, k);
    }
    D[i] = d > 0.0 ? d : 1.0;
}

// right-hand sides.  heat: 1 at the sources (level 0).  Poisson: per vertex
// the sum over its faces, visited through its one-ring edges (each face is
// met twice, by its two edges at the vertex, hence the half); 0 where fixed.
__global__ void k_cg_rhs(int n, int op, const int32_t* __restrict__ level, const uint8_t* __restrict__ fixed,
                         const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ csr_edge,
                         const int32_t* __restrict__ ef, const int32_t* __restrict__ tri,
                         const double* __restrict__ px, const double* __restrict__ py, const double* __restrict__ pz,
                         const float* __restrict__ h, double* __restrict__ b) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (op == CG_HEAT) {
        b[i] = level[i] == 0 ? 1.0 : 0.0;
        return;
    }
    if (fixed[i]) {
        b[i] = 0.0;
        return;
    }
    double acc = 0.0;
    for (int k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
        const int e = csr_edge[k];
        for (int side = 0; side < 2; ++side) {
            const int f = ef[2 * e + side];
            if (f < 0) continue;
            int c = 0;
            while (c < 2 && tri[3 * f + c] != i) ++c;
            const int a = tri[3 * f + c], bb = tri[3 * f + (c + 1) % 3], cc = tri[3 * f + (c + 2) % 3];
            const double hf[3] = {(double)h[3 * f], (double)h[3 * f + 1], (double)h[3 * f + 2]};
            if (op == CG_FACE) {
                // A_f grad phi_a . h = (N x e_a) . h / 2, e_a = p_c - p_b, N the unit normal
                const double u[3] = {px[bb] - px[a], py[bb] - py[a], pz[bb] - pz[a]};
                const double v[3] = {px[cc] - px[a], py[cc] - py[a], pz[cc] - pz[a]};
                double nrm[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
                const double ln = sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
                nrm[0] /= ln;
                nrm[1] /= ln;
                nrm[2] /= ln;
                const double ea[3] = {v[0] - u[0], v[1] - u[1], v[2] - u[2]};
                const double g[3] = {nrm[1] * ea[2] - nrm[2] * ea[1], nrm[2] * ea[0] - nrm[0] * ea[2],
                                     nrm[0] * ea[1] - nrm[1] * ea[0]};
                acc += 0.5 * (g[0] * hf[0] + g[1] * hf[1] + g[2] * hf[2]);
            } else {
                const double q[3] = {2.0 * px[a] - px[bb] - px[cc], 2.0 * py[a] - py[bb] - py[cc],
                                     2.0 * pz[a] - pz[bb] - pz[cc]};
                acc += q[0] * hf[0] + q[1] * hf[1] + q[2] * hf[2];
            }
        }
    }
    b[i] = 0.5 * acc;
}

// x = 0, r = b, z = r / D, p = z; partial sums of r.z, r.r and b.b
__global__ void __launch_bounds__(kBlockC) k_cg_init(int n, const double* __restrict__ b,
                                                     const double* __restrict__ D, double* __restrict__ x,
                                                     double* __restrict__ r, double* __restrict__ z,
                                                     double* __restrict__ p, double* __restrict__ partial,
                                                     int stride) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double v[3] = {0.0, 0.0, 0.0};
    if (i < n) {
        const double bi = b[i], zi = bi / D[i];
        x[i] = 0.0;
        r[i] = bi;
        z[i] = zi;
        p[i] = zi;
        v[0] = bi * zi;
        v[1] = bi * bi;
        v[2] = bi * bi;
    }
    block_sums<3>(v, partial, stride);
}

// q = A p (0 on fixed rows); partial sums of p.q
__global__ void __launch_bounds__(kBlockC) k_cg_spmv(int n, CgOp M, const uint8_t* __restrict__ fixed,
                                                     const double* __restrict__ p, double* __restrict__ q,
                                                     double* __restrict__ partial, int stride) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double v[1] = {0.0};
    if (i < n) {
        double qi = 0.0;
        if (!fixed[i]) {
            double d;
            qi = apply_row(M, i, p, &d);
        }
        q[i] = qi;
        v[0] = p[i] * qi;
    }
    block_sums<1>(v, partial, stride);
}

// alpha = rz / pq; x += alpha p; r -= alpha q; z = r / D (0 where fixed);
// partial sums of the new r.z and r.r
__global__ void __launch_bounds__(kBlockC) k_cg_update(int n, int it, const uint8_t* __restrict__ fixed,
                                                       const double* __restrict__ D, const double* __restrict__ p,
                                                       const double* __restrict__ q, double* __restrict__ x,
                                                       double* __restrict__ r, double* __restrict__ z,
                                                       const double* __restrict__ scal, double* __restrict__ partial,
                                                       int stride) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const double rz = scal[(it & 1) ? S_RZ1 : S_RZ0], pq = scal[S_PQ];
    const double alpha = pq > 0.0 ? rz / pq : 0.0;
    double v[2] = {0.0, 0.0};
    if (i < n) {
        const double xi = fma(alpha, p[i], x[i]);
        const double ri = fma(-alpha, q[i], r[i]);
        const double zi = fixed[i] ? 0.0 : ri / D[i];
        x[i] = xi;
        r[i] = ri;
        z[i] = zi;
        v[0] = ri * zi;
        v[1] = ri * ri;
    }
    block_sums<2>(v, partial, stride);
}

// beta = rz_new / rz_old; p = z + beta p
__global__ void k_cg_pupdate(int n, int it, const double* __restrict__ z, double* __restrict__ p,
                             const double* __restrict__ scal) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double rz_old = scal[(it & 1) ? S_RZ1 : S_RZ0], rz_new = scal[(it & 1) ? S_RZ0 : S_RZ1];
    const double beta = rz_old > 0.0 ? rz_new / rz_old : 0.0;
    p[i] = fma(beta, p[i], z[i]);
}

// Poisson outputs: +inf where no source reaches
__global__ void k_cg_mark_unreached(int n, const int32_t* __restrict__ level, double* __restrict__ x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && level[i] < 0) x[i] = INFINITY;
}

__global__ void k_cg_fixed(int n, int op, const int32_t* __restrict__ level, uint8_t* __restrict__ fixed) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) fixed[i] = op == CG_HEAT ? 0 : (level[i] <= 0 ? 1 : 0);
}

// true residual of the heat system for a given u: partial sums of
// ((A - t L_c) u - u_0)_i^2
__global__ void __launch_bounds__(kBlockC) k_heat_residual(int n, CgOp M, const int32_t* __restrict__ level,
                                                           const double* __restrict__ u, double* __restrict__ partial,
                                                           int stride) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double v[1] = {0.0};
    if (i < n) {
        double d;
        const double y = apply_row(M, i, u, &d);
        const double ri = y - (level[i] == 0 ? 1.0 : 0.0);
        v[0] = ri * ri;
    }
    block_sums<1>(v, partial, stride);
}

__global__ void k_exp_if_log(int n, const double* __restrict__ in, int is_log, double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = is_log ? exp(in[i]) : in[i];
}

static CgOp make_op(Mesh& m, Work& w, int op) {
    CgOp M;
    M.op = op;
    M.row_ptr = m.row_ptr.p;
    M.col = m.col.p;
    M.csr_edge = m.csr_edge.p;
    M.ef = m.ef.p;
    M.comp = m.comp_v.p;
    M.theta = m.theta.p;
    M.Av = m.Av.p;
    M.sum_theta = m.sum_theta.p;
    M.tcomp = w.tcomp.p;
    return M;
}

static void upload_t(Mesh& m, Work& w, const std::vector<double>& tc, hipStream_t s) {
    w.tcomp.alloc(tc.size());
    HG_CHECK_HIP(hipMemcpyAsync(w.tcomp.p, tc.data(), tc.size() * sizeof(double), hipMemcpyHostToDevice, s));
    HG_CHECK_HIP(hipStreamSynchronize(s));   // tc is the caller's host vector
    (void)m;
}

CgResult run_cg(Mesh& m, Work& w, int op, const std::vector<int32_t>& src_internal, const std::vector<double>& tc,
                const float* h_internal, int max_iters, double tol, hipStream_t s) {
    const int n = (int)m.nv;
    const int nb = grid_for(n, kBlockC);
    auto& C = w.cg;
    C.x.alloc(n);
    C.r.alloc(n);
    C.z.alloc(n);
    C.p.alloc(n);
    C.q.alloc(n);
    C.D.alloc(n);
    C.b.alloc(n);
    C.fixed.alloc(n);
    C.partial.alloc((size_t)3 * nb);
    C.scal.alloc(S_N);
    w.ensure_pinned();
    run_bfs(m, w, src_internal, s);
    if (op == CG_HEAT) upload_t(m, w, tc, s);
    const CgOp M = make_op(m, w, op);
    const int g = nb;
    hipLaunchKernelGGL(k_cg_fixed, dim3(g), dim3(kBlockC), 0, s, n, op, w.level.p, C.fixed.p);
    hipLaunchKernelGGL(k_cg_diag, dim3(g), dim3(kBlockC), 0, s, n, M, C.fixed.p, C.D.p);
    hipLaunchKernelGGL(k_cg_rhs, dim3(g), dim3(kBlockC), 0, s, n, op, w.level.p, C.fixed.p, m.row_ptr.p,
                       m.csr_edge.p, m.ef.p, m.tri.p, m.px.p, m.py.p, m.pz.p, h_internal, C.b.p);
    hipLaunchKernelGGL(k_cg_init, dim3(g), dim3(kBlockC), 0, s, n, C.b.p, C.D.p, C.x.p, C.r.p, C.z.p, C.p.p,
                       C.partial.p, nb);
    hipLaunchKernelGGL(k_cg_reduce, dim3(1), dim3(kBlockC), 0, s, C.partial.p, nb, nb, 3, (int)S_RZ0, (int)S_RR,
                       (int)S_BB, C.scal.p);
    HG_CHECK_HIP(hipGetLastError());
    CgResult res;
    hipEvent_t e0, e1;
    HG_CHECK_HIP(hipEventCreate(&e0));
    HG_CHECK_HIP(hipEventCreate(&e1));
    HG_CHECK_HIP(hipEventRecord(e0, s));
    double hs[S_N];
    auto read_scal = [&] {
        HG_CHECK_HIP(hipMemcpyAsync(w.pinned, C.scal.p, S_N * sizeof(double), hipMemcpyDeviceToHost, s));
        HG_CHECK_HIP(hipStreamSynchronize(s));
        std::copy(w.pinned, w.pinned + S_N, hs);
    };
    int it = 0;
    try {
        read_scal();
        const double bb = hs[S_BB];
        res.res_abs0 = std::sqrt(bb);
        if (bb > 0.0) {
            while (it < max_iters) {
                hipLaunchKernelGGL(k_cg_spmv, dim3(g), dim3(kBlockC), 0, s, n, M, C.fixed.p, C.p.p, C.q.p,
                                   C.partial.p, nb);
                hipLaunchKernelGGL(k_cg_reduce, dim3(1), dim3(kBlockC), 0, s, C.partial.p, nb, nb, 1, (int)S_PQ, 0,
                                   0, C.scal.p);
                hipLaunchKernelGGL(k_cg_update, dim3(g), dim3(kBlockC), 0, s, n, it, C.fixed.p, C.D.p, C.p.p, C.q.p,
                                   C.x.p, C.r.p, C.z.p, C.scal.p, C.partial.p, nb);
                hipLaunchKernelGGL(k_cg_reduce, dim3(1), dim3(kBlockC), 0, s, C.partial.p, nb, nb, 2,
                                   (it & 1) ? (int)S_RZ0 : (int)S_RZ1, (int)S_RR, 0, C.scal.p);
                hipLaunchKernelGGL(k_cg_pupdate, dim3(g), dim3(kBlockC), 0, s, n, it, C.z.p, C.p.p, C.scal.p);
                HG_CHECK_HIP(hipGetLastError());
                ++it;
                if (tol > 0.0 && (it % kCgCheck == 0 || it == max_iters)) {
                    read_scal();
                    if (std::sqrt(hs[S_RR] / bb) <= tol) {
                        res.converged = true;
                        break;
                    }
                }
            }
        } else {
            res.converged = true;
        }
        HG_CHECK_HIP(hipEventRecord(e1, s));
        HG_CHECK_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        HG_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
        res.ms = ms;
        read_scal();
        res.iters = it;
        res.res_abs = std::sqrt(std::max(hs[S_RR], 0.0));
        res.res_rel = bb > 0.0 ? res.res_abs / std::sqrt(bb) : 0.0;
        if (tol > 0.0 && res.res_rel <= tol) res.converged = true;
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (op != CG_HEAT)
        hipLaunchKernelGGL(k_cg_mark_unreached, dim3(g), dim3(kBlockC), 0, s, n, w.level.p, C.x.p);
    HG_CHECK_HIP(hipGetLastError());
    return res;
}

double heat_residual(Mesh& m, Work& w, const std::vector<int32_t>& src_internal, const std::vector<double>& tc,
                     const double* u_internal, bool is_log, hipStream_t s) {
    const int n = (int)m.nv;
    const int nb = grid_for(n, kBlockC);
    auto& C = w.cg;
    C.q.alloc(n);
    C.partial.alloc((size_t)3 * nb);
    C.scal.alloc(S_N);
    w.ensure_pinned();
    run_bfs(m, w, src_internal, s);
    upload_t(m, w, tc, s);
    const CgOp M = make_op(m, w, CG_HEAT);
    hipLaunchKernelGGL(k_exp_if_log, dim3(nb), dim3(kBlockC), 0, s, n, u_internal, is_log ? 1 : 0, C.q.p);
    hipLaunchKernelGGL(k_heat_residual, dim3(nb), dim3(kBlockC), 0, s, n, M, w.level.p, C.q.p, C.partial.p, nb);
    hipLaunchKernelGGL(k_cg_reduce, dim3(1), dim3(kBlockC), 0, s, C.partial.p, nb, nb, 1, (int)S_RR, 0, 0,
                       C.scal.p);
    HG_CHECK_HIP(hipGetLastError());
    HG_CHECK_HIP(hipMemcpyAsync(w.pinned, C.scal.p + S_RR, sizeof(double), hipMemcpyDeviceToHost, s));
    HG_CHECK_HIP(hipStreamSynchronize(s));
    return std::sqrt(std::max(*w.pinned, 0.0));
}

}  // namespace hg

using namespace hg;

namespace {
std::vector<double> cg_times(const Mesh& m, double t) {
    std::vector<double> tc((size_t)std::max(1, m.n_comp));
    for (auto& x : tc) x = (t > 0.0 && std::isfinite(t)) ? t : m.hbar * m.hbar;
    return tc;
}
void fill_cg_info(const CgResult& r, hg_cg_info* info) {
    if (!info) return;
    std::memset(info, 0, sizeof(*info));
    info->iters = r.iters;
    info->converged = r.converged ? 1 : 0;
    info->res_rel = r.res_rel;
    info->res_abs = r.res_abs;
    info->res_abs0 = r.res_abs0;
    info->ms = (float)r.ms;
}
}  // namespace

extern "C" {

hg_status hg_cg_diffuse(hg_mesh_t mesh, const int32_t* src, int32_t nsrc, double t, int32_t max_iters, double tol,
                        double* u_dev, void* stream, hg_cg_info* info) {
    return guarded([&]() -> hg_status {
        if (!mesh || !u_dev) return fail(HG_E_INVALID_ARG, "null argument");
        if (max_iters < 0 || !(tol >= 0.0)) return fail(HG_E_INVALID_ARG, "max_iters and tol must be >= 0");
        auto* m = reinterpret_cast<Mesh*>(mesh);
        hipStream_t s = (hipStream_t)stream;
        auto si = map_sources(*m, src, nsrc);
        CgResult r = run_cg(*m, m->w, CG_HEAT, si, cg_times(*m, t), nullptr, max_iters, tol, s);
        scatter_vertices_to_user_d(*m, m->w.cg.x.p, u_dev, s);
        HG_CHECK_HIP(hipStreamSynchronize(s));
        fill_cg_info(r, info);
        return (tol > 0.0 && !r.converged) ? fail(HG_E_NOT_CONVERGED, "CG iteration cap reached") : HG_OK;
    });
}

hg_status hg_cg_poisson(hg_mesh_t mesh, int32_t form, const float* h_dev, const int32_t* src, int32_t nsrc,
                        int32_t max_iters, double tol, double* d_dev, void* stream, hg_cg_info* info) {
    return guarded([&]() -> hg_status {
        if (!mesh || !h_dev || !d_dev) return fail(HG_E_INVALID_ARG, "null argument");
        if (form != HG_FORM_FACE && form != HG_FORM_EDGE)
            return fail(HG_E_INVALID_ARG, "form must be HG_FORM_FACE or HG_FORM_EDGE");
        if (max_iters < 0 || !(tol >= 0.0)) return fail(HG_E_INVALID_ARG, "max_iters and tol must be >= 0");
        auto* m = reinterpret_cast<Mesh*>(mesh);
        if (m->intrinsic) return fail(HG_E_INVALID_ARG, "hg_cg_poisson needs an extrinsic mesh");
        hipStream_t s = (hipStream_t)stream;
        auto si = map_sources(*m, src, nsrc);
        m->w.h.alloc((size_t)3 * m->nf);
        gather_faces_to_internal(*m, h_dev, m->w.h.p, s);
        CgResult r = run_cg(*m, m->w, form == HG_FORM_FACE ? CG_FACE : CG_EDGE, si, cg_times(*m, 0.0), m->w.h.p,
                            max_iters, tol, s);
        scatter_vertices_to_user_d(*m, m->w.cg.x.p, d_dev, s);
        HG_CHECK_HIP(hipStreamSynchronize(s));
        fill_cg_info(r, info);
        return (tol > 0.0 && !r.converged) ? fail(HG_E_NOT_CONVERGED, "CG iteration cap reached") : HG_OK;
    });
}

hg_status hg_heat_residual(hg_mesh_t mesh, const int32_t* src, int32_t nsrc, double t, const double* u_dev,
                           int32_t is_log, double* e1, void* stream) {
    return guarded([&]() -> hg_status {
        if (!mesh || !u_dev || !e1) return fail(HG_E_INVALID_ARG, "null argument");
        auto* m = reinterpret_cast<Mesh*>(mesh);
        hipStream_t s = (hipStream_t)stream;
        auto si = map_sources(*m, src, nsrc);
        m->w.cg.x.alloc(m->nv);
        gather_vertices_to_internal_d(*m, u_dev, m->w.cg.x.p, s);
        *e1 = heat_residual(*m, m->w, si, cg_times(*m, t), m->w.cg.x.p, is_log != 0, s);
        return HG_OK;
    });
}

}  // extern "C"
