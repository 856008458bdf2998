// Heat diffusion (A - t L_c) u = u_0 (Eq. 4) by sweeps of the update Eq. 7,
//     u_j <- (u_0(j) + t sum_k theta_jk u_k) / (A_j + t sum_k theta_jk),
// with u_0 = 1 at every source.  The paper sweeps the breadth-first sets in
// order on a CPU; here every vertex is updated from the previous sweep's
// values (Jacobi), which needs no ordering and is bit-for-bit deterministic;
// the fixed point is the same discrete solution.
//
// Range.  For t ~ hbar^2 the solution falls by ~e^-1 per ring of vertices
// and leaves the FP64 range after ~700 rings.  Each value is therefore kept
// as u_j = v_j * 2^e_j (FP64 mantissa v_j in [1, 2), int32 exponent e_j).
// An update first takes the largest exponent m among its non-zero
// neighbours, scales every neighbour by the exact power of two 2^(e_k - m)
// (ldexp), sums, and renormalises; rounding is that of plain FP64 on
// u * 2^-m, and no value can overflow or underflow.  (Mantissas keep their
// sign: with obtuse triangles some theta_jk < 0 and iterates may dip below
// zero before converging.)
#include <climits>
#include <cmath>

#include "hgeo_internal.h"

namespace hg {

constexpr int kBlockD = 256;

__device__ inline double block_max(double v) {
    __shared__ double sh[kBlockD / 64];
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = sh[0];
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = fmax(r, sh[i]);
        v = r;
    }
    __syncthreads();
    return v;
}

// 1 / (A_j + t sum_k theta_jk), and the initial state (1 at sources, else 0).
__global__ void k_diff_init(int nv, const double* tcomp, const int32_t* comp, const double* Av,
                            const double* sum_theta, const int32_t* level, double* invD, double* v, int32_t* e) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nv) return;
    invD[j] = 1.0 / (Av[j] + tcomp[comp[j]] * sum_theta[j]);
    v[j] = level[j] == 0 ? 1.0 : 0.0;
    e[j] = 0;
}

// One Jacobi sweep.  res: largest relative change |u_new - u_old| / u_new
// over reachable vertices (1 for a vertex that is still 0 or just reached).
__global__ void __launch_bounds__(kBlockD) k_diff_sweep(int nv, const double* __restrict__ tcomp,
                                                        const int32_t* __restrict__ comp,
                                                        const int32_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ col,
                                                        const double* __restrict__ theta,
                                                        const double* __restrict__ invD,
                                                        const int32_t* __restrict__ level,
                                                        const double* __restrict__ vin,
                                                        const int32_t* __restrict__ ein, double* __restrict__ vout,
                                                        int32_t* __restrict__ eout, int want_res,
                                                        double* __restrict__ partial) {
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int j = b * blockDim.x + threadIdx.x;
    double res = 0.0;
    if (j < nv) {
        const int lj = level[j];
        if (lj < 0) {
            vout[j] = 0.0;
            eout[j] = 0;
        } else {
            const int k0 = row_ptr[j], k1 = row_ptr[j + 1];
            int m = (lj == 0) ? 0 : INT_MIN;
            for (int k = k0; k < k1; ++k) {
                const int c = col[k];
                if (vin[c] != 0.0) m = max(m, ein[c]);
            }
            if (m == INT_MIN) {
                vout[j] = 0.0;
                eout[j] = 0;
                res = 1.0;
            } else {
                double acc = 0.0;
                for (int k = k0; k < k1; ++k) {
                    const int c = col[k];
                    acc += theta[k] * ldexp(vin[c], ein[c] - m);
                }
                double y = tcomp[comp[j]] * acc;
                if (lj == 0) y += ldexp(1.0, -m);
                y *= invD[j];
                if (y == 0.0) {
                    // possible transiently where some theta_jk < 0
                    vout[j] = 0.0;
                    eout[j] = 0;
                    res = 1.0;
                } else {
                    const int ex = ilogb(y);
                    const double vn = ldexp(y, -ex);
                    const int en = m + ex;
                    vout[j] = vn;
                    eout[j] = en;
                    if (want_res) {
                        const double vo = vin[j];
                        if (vo == 0.0) {
                            res = 1.0;
                        } else {
                            const double old = ldexp(vo, ein[j] - en);
                            res = fabs(vn - old) / fabs(vn);
                        }
                    }
                }
            }
        }
    }
    if (want_res) {
        res = block_max(res);
        if (threadIdx.x == 0) partial[blockIdx.x] = res;
    }
}

__global__ void k_diff_logu(int nv, const double* v, const int32_t* e, double* logu) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nv) return;
    double x = v[j];
    logu[j] = x > 0.0 ? log(x) + (double)e[j] * 0.69314718055994530942 : -INFINITY;
}

static DiffusionResult run_diffusion_jacobi(Mesh& m, Work& w, const hg_opts& o, hipStream_t s);

__global__ void k_tile_t(int nt, const int32_t* tile_comp, const double* tcomp, double* tile_t) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nt) tile_t[p] = tcomp[tile_comp[p]];
}

// Schedule choice: LDS-tiled passes (default when every tile's valence fits)
// or plain global Jacobi sweeps.  Both start from u = 1 at the sources and 0
// elsewhere and stop on the largest relative change of u.
DiffusionResult run_diffusion(Mesh& m, Work& w, const std::vector<int32_t>& src, const std::vector<double>& t,
                              const hg_opts& o, hipStream_t s) {
    (void)src;   // sources are the level-0 vertices of the preceding BFS
    const int nv = (int)m.nv;
    w.v0.alloc(nv);
    w.v1.alloc(nv);
    w.e0.alloc(nv);
    w.e1.alloc(nv);
    w.invD.alloc(nv);
    const int grid = grid_for(nv, kBlockD);
    if ((int)t.size() != m.n_comp) throw Error{HG_E_INVALID_ARG, "one diffusion time per component expected"};
    w.tcomp.upload(t, s);
    w.tile_t.alloc(std::max(1, m.n_patches));
    hipLaunchKernelGGL(k_tile_t, dim3(grid_for(m.n_patches, kBlockD)), dim3(kBlockD), 0, s, m.n_patches,
                       m.tile_comp.p, w.tcomp.p, w.tile_t.p);
    hipLaunchKernelGGL(k_diff_init, dim3(grid), dim3(kBlockD), 0, s, nv, w.tcomp.p, m.comp_v.p, m.Av.p,
                       m.sum_theta.p, w.level.p, w.invD.p, w.v0.p, w.e0.p);
    HG_CHECK_HIP(hipGetLastError());
    const int sched = o.diffusion_schedule != 0 ? o.diffusion_schedule : m.tuned_schedule;
    const bool patch = sched == 2 || sched == 3 || (sched == 0 && patch_supported(m));
    if (patch) {
        if (!patch_supported(m)) throw Error{HG_E_INVALID_ARG, "tiled schedule needs valence <= 16"};
        const int inner = o.inner_sweeps > 0 ? o.inner_sweeps : (m.tuned_inner > 0 ? m.tuned_inner : 32);
        const int rings =
            o.overlap_rings > 0 ? o.overlap_rings : (m.tuned_rings > 0 ? m.tuned_rings : kAutoOverlapRings);
        return run_diffusion_patch(m, w, o, inner, s, sched == 3 ? rings : 0);
    }
    return run_diffusion_jacobi(m, w, o, s);
}

static DiffusionResult run_diffusion_jacobi(Mesh& m, Work& w, const hg_opts& o, hipStream_t s) {
    const int nv = (int)m.nv;
    const int grid = grid_for(nv, kBlockD);
    if ((int)w.partial.n < grid + 8) w.partial.alloc((size_t)grid + 8);
    DiffusionResult r;
    const int check = std::max(1, o.check_every);
    double* va = w.v0.p;
    double* vb = w.v1.p;
    int32_t* ea = w.e0.p;
    int32_t* eb = w.e1.p;
    // algorithmic bytes of one sweep: CSR (row_ptr, col, theta), 1/D, level,
    // own (v, e) read once, (v, e) written
    r.bytes_per_pass = (uint64_t)4 * (nv + 1) + (uint64_t)24 * m.ne + (uint64_t)36 * nv;
    RunTimer rt;
    int run_len = 0;
    for (int it = 1; it <= o.max_sweeps; ++it) {
        const bool want = (it % check) == 0 || it == o.max_sweeps;
        if (!rt.open) {
            rt.start(s);
            run_len = 0;
        }
        hipLaunchKernelGGL(k_diff_sweep, dim3(grid), dim3(kBlockD), 0, s, nv, w.tcomp.p, m.comp_v.p, m.row_ptr.p,
                           m.col.p, m.theta.p,
                           w.invD.p, w.level.p, va, ea, vb, eb, want ? 1 : 0, w.partial.p);
        HG_CHECK_HIP(hipGetLastError());
        ++run_len;
        std::swap(va, vb);
        std::swap(ea, eb);
        r.sweeps = it;
        if (want) {
            r.kernel_ms += rt.stop(s);
            r.timed_launches += run_len;
            r.res = reduce_partials(m, w, grid, true, s);
            if (r.res <= o.tol_u) {
                r.converged = true;
                break;
            }
        }
    }
    r.passes = r.sweeps;
    // the current state lives in (va, ea); make it (v0, e0)
    if (va != w.v0.p) {
        HG_CHECK_HIP(hipMemcpyAsync(w.v0.p, va, (size_t)nv * sizeof(double), hipMemcpyDeviceToDevice, s));
        HG_CHECK_HIP(hipMemcpyAsync(w.e0.p, ea, (size_t)nv * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
    return r;
}

void diffusion_logu(Mesh& m, Work& w, hipStream_t s) {
    w.logu.alloc(m.nv);
    hipLaunchKernelGGL(k_diff_logu, dim3(grid_for(m.nv, kBlockD)), dim3(kBlockD), 0, s, (int)m.nv, w.v0.p,
                       w.e0.p, w.logu.p);
    HG_CHECK_HIP(hipGetLastError());
}

}  // namespace hg
