// Normalisation (Eq. 3), edge targets (Eq. 18) and the two ADMM solvers of
// the gradient optimisation: face form (Sec. 3.2) and edge form (Sec. 4.1).
//
// Both solvers run the paper's iterations, optionally over-relaxed with
// alpha (the standard over-relaxed ADMM of the ADMM survey the paper cites;
// alpha = 1 is the paper's iteration, the fixed point does not depend on it),
// with the state folded so that one fused kernel per iteration suffices:
//
// Edge form.  Per face slot keep zeta = lambda + mu w (of the current
// iteration); then x_e = (sum_h h_e + sum_slots zeta) / (|H_e| (1 + mu))
// (Eq. 21), lambda = zeta - mu x, and the next W-update projects
// x - lambda/mu = 2x - zeta/mu.  One iteration per face f and slot k:
//     x_k   = (S_e + zeta_e0 + zeta_e1) / (|H_e| (1 + mu))
//     w_f   = (I - q q^T/3)(2 x_f - zeta_f / mu)
//     zeta' = zeta_f + mu alpha (w_f - x_f)
// (zeta = lambda + mu w_hat with w_hat = alpha w + (1 - alpha) x.)
// Starting from zeta = mu * (mean target) reproduces the paper's
// initialisation (lambda = 0, x = mean of targets).
// Layout: zeta is kept per face slot (3f + k), with a copy of S_e per slot
// and the slot of the edge's other face ("twin", -1 on the boundary), so a
// face reads and writes its three slots contiguously and gathers only the
// twins' zeta: the iteration streams 49 bytes per face.
//
// Face form.  Per auxiliary copy k of face i keep z = y + lambda/(mu alpha_i);
// then q_k = g_i - lambda_k/(mu alpha_i) = 2 g_i - z_k, the Y-update gives
// y_k, the new z_k = z_k + alpha (y_k - g_i), and the G-update is
// g_i = (2 h_i + mu sum_k z_k) / (2 + mu |Y(i)|).  Each face computes its own
// copies' Y-update (it reads the neighbour's g and z across the edge), so
// one kernel per face performs Y, G and lambda updates.  z = h initially.
// Layout, as in the edge form: the copies per face slot (3f + k), with each
// slot's unit edge vector and neighbour weight A_nb / (A_own + A_nb) (sgeo)
// and its twin slot, so a face reads and writes its own data contiguously
// and gathers only the neighbours' g and copies: 168 bytes per face.
//
// g, z and zeta are double-buffered (Jacobi semantics, deterministic).
// Residuals are those of the paper, recovered exactly from two consecutive
// states (see k_resid_edge / k_resid_face).
#include <cmath>

#include "hgeo_internal.h"

namespace hg {

constexpr int kBlockA = 256;

__device__ inline double block_sum2(double v) {
    __shared__ double sh[kBlockA / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = sh[0];
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
        v = r;
    }
    __syncthreads();
    return v;
}

// ------------------------------------------------------------ normalisation
// h_f = -grad u / |grad u| from u = v 2^e; the three values are first scaled
// by 2^-max(e) (the direction does not depend on the scale).  grad u is
// proportional to sum_i u_i (n x e_i), n = (p1-p0)x(p2-p0), e_i the CCW edge
// opposite corner i.
__global__ void k_normalize(int nf, const int32_t* tri, const double* px, const double* py, const double* pz,
                            const double* floc, const double* v, const int32_t* e, float* h) {
    int f = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    int id[3] = {tri[3 * f], tri[3 * f + 1], tri[3 * f + 2]};
    double vv[3];
    int ee[3];
    int m = -0x7fffffff;
    for (int k = 0; k < 3; ++k) {
        vv[k] = v[id[k]];
        ee[k] = e[id[k]];
        if (vv[k] != 0.0) m = max(m, ee[k]);
    }
    double p[3][3];
    if (floc) {   // intrinsic: the face's own plane, h in that frame (z = 0)
        p[0][0] = p[0][1] = p[0][2] = 0.0;
        p[1][0] = floc[3 * f];
        p[1][1] = p[1][2] = 0.0;
        p[2][0] = floc[3 * f + 1];
        p[2][1] = floc[3 * f + 2];
        p[2][2] = 0.0;
    } else {
        for (int k = 0; k < 3; ++k) {
            p[k][0] = px[id[k]];
            p[k][1] = py[id[k]];
            p[k][2] = pz[id[k]];
        }
    }
    double a[3], b[3], n[3];
    for (int c = 0; c < 3; ++c) {
        a[c] = p[1][c] - p[0][c];
        b[c] = p[2][c] - p[0][c];
    }
    n[0] = a[1] * b[2] - a[2] * b[1];
    n[1] = a[2] * b[0] - a[0] * b[2];
    n[2] = a[0] * b[1] - a[1] * b[0];
    double g[3] = {0.0, 0.0, 0.0};
    if (m != -0x7fffffff) {
        for (int k = 0; k < 3; ++k) {
            if (vv[k] == 0.0) continue;
            double wk = ldexp(vv[k], ee[k] - m);
            const double* pa = p[(k + 1) % 3];
            const double* pb = p[(k + 2) % 3];
            double ed[3] = {pb[0] - pa[0], pb[1] - pa[1], pb[2] - pa[2]};
            g[0] += wk * (n[1] * ed[2] - n[2] * ed[1]);
            g[1] += wk * (n[2] * ed[0] - n[0] * ed[2]);
            g[2] += wk * (n[0] * ed[1] - n[1] * ed[0]);
        }
    }
    double nrm = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    float hx = 0.f, hy = 0.f, hz = 0.f;
    if (nrm > 0.0) {
        hx = (float)(-g[0] / nrm);
        hy = (float)(-g[1] / nrm);
        hz = (float)(-g[2] / nrm);
    }
    h[3 * f] = hx;
    h[3 * f + 1] = hy;
    h[3 * f + 2] = hz;
}

// sum over the incident faces of h_f . (p_head - p_tail) (Eq. 18), per edge.
__global__ void k_edge_targets(int ne, const int32_t* ev, const int32_t* ef, const double* px, const double* py,
                               const double* pz, const float* h, float* sumz) {
    int e = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    int a = ev[2 * e], b = ev[2 * e + 1];
    double d[3] = {px[b] - px[a], py[b] - py[a], pz[b] - pz[a]};
    double s = 0.0;
    for (int q = 0; q < 2; ++q) {
        int f = ef[2 * e + q];
        if (f < 0) continue;
        s += (double)h[3 * f] * d[0] + (double)h[3 * f + 1] * d[1] + (double)h[3 * f + 2] * d[2];
    }
    sumz[e] = (float)s;
}

// Intrinsic meshes: per edge, the sum over its faces of h_f . (P_head -
// P_tail) with the corners P in each face's own frame (Eq. 18).
__global__ void k_edge_targets_local(int ne, const int32_t* ef, const uint32_t* fslot, const uint8_t* fsign,
                                     const double* floc, const float* h, float* sumz) {
    int e = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    double s = 0.0;
    for (int q = 0; q < 2; ++q) {
        int f = ef[2 * e + q];
        if (f < 0) continue;
        const double P[3][2] = {{0.0, 0.0}, {floc[3 * f], 0.0}, {floc[3 * f + 1], floc[3 * f + 2]}};
        for (int k = 0; k < 3; ++k) {
            if (slot_edge(fslot[3 * f + k]) != e) continue;
            const double dx = P[(k + 1) % 3][0] - P[k][0], dy = P[(k + 1) % 3][1] - P[k][1];
            const double z = (double)h[3 * f] * dx + (double)h[3 * f + 1] * dy;
            s += ((fsign[f] >> k) & 1) ? z : -z;   // the slot runs tail -> head, or the reverse
        }
    }
    sumz[e] = (float)s;
}

void run_normalize(Mesh& m, Work& w, hipStream_t s) {
    w.h.alloc((size_t)3 * m.nf);
    hipLaunchKernelGGL(k_normalize, dim3(grid_for(m.nf, kBlockA)), dim3(kBlockA), 0, s, (int)m.nf, m.tri.p, m.px.p,
                       m.py.p, m.pz.p, m.intrinsic ? m.floc.p : nullptr, w.v0.p, w.e0.p, w.h.p);
    HG_CHECK_HIP(hipGetLastError());
}

// (v, e) from a caller log u, then normalise (stage entry point).
__global__ void k_logu_to_ve(int nv, const int32_t* perm_v, const double* logu_user, double* v, int32_t* e) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nv) return;
    double l = logu_user[perm_v[j]];
    if (!(l > -INFINITY)) {
        v[j] = 0.0;
        e[j] = 0;
        return;
    }
    double ex = floor(l / 0.69314718055994530942);
    e[j] = (int)ex;
    v[j] = exp(l - ex * 0.69314718055994530942);
}

void normalize_from_logu(Mesh& m, Work& w, const double* logu_user, hipStream_t s) {
    w.v0.alloc(m.nv);
    w.e0.alloc(m.nv);
    hipLaunchKernelGGL(k_logu_to_ve, dim3(grid_for(m.nv, kBlockA)), dim3(kBlockA), 0, s, (int)m.nv, m.perm_v.p,
                       logu_user, w.v0.p, w.e0.p);
    HG_CHECK_HIP(hipGetLastError());
    run_normalize(m, w, s);
}

// ---------------------------------------------------------------- edge form
__global__ void k_zeta_init(int ne, const int32_t* h01, const float* sumz, float mu, float* zeta, float* sumd) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const int h0 = h01[2 * e], h1 = h01[2 * e + 1];
    float nh = h1 >= 0 ? 2.f : 1.f;
    float z = mu * (sumz[e] / nh);
    zeta[h0] = z;
    sumd[h0] = sumz[e];
    if (h1 >= 0) {
        zeta[h1] = z;
        sumd[h1] = sumz[e];
    }
}


// One folded iteration of a face from its three copies zo and per slot the
// twin's copy tz and target sum S, with c = 1 / (2 (1 + mu)) and the sign q
// (Eq. 20); rmu = 1 / mu.  The X-update x = (S + zo + tz) c covers both
// kinds of edge: an interior edge has |H_e| = 2; a boundary slot passes its
// own copy as tz and 2 S, which gives (S + zo) / (1 + mu) up to rounding.
// Contraction is off and the fused operations are written out, so every
// kernel that inlines this rounds the same way.
__device__ inline void edge_face_update(const float zo[3], const float tz[3], const float S[3], const float q[3],
                                        float c, float rmu, float mu_relax, float zn[3]) {
#pragma clang fp contract(off)
    float x[3], v[3];
    float qv = 0.f;
    for (int k = 0; k < 3; ++k) {
        x[k] = (S[k] + zo[k] + tz[k]) * c;
        v[k] = fmaf(-zo[k], rmu, x[k] + x[k]);
        qv += q[k] * v[k];   // q = +-1: exact
    }
    qv *= (1.f / 3.f);
    for (int k = 0; k < 3; ++k) {
        const float w = fmaf(-qv, q[k], v[k]);
        zn[k] = fmaf(mu_relax, w - x[k], zo[k]);
    }
}

__device__ inline void admm_edge_face(int f, const int32_t* __restrict__ twin, const uint8_t* __restrict__ fsign,
                                      const float* __restrict__ sumd, const float* __restrict__ zin,
                                      float* __restrict__ zout, float rmu, float c, float mu_relax) {
    float zo[3], tz[3], S[3], q[3], zn[3];
    int tw[3];
    for (int k = 0; k < 3; ++k) {
        tw[k] = twin[3 * f + k];
        zo[k] = zin[3 * f + k];
    }
    const uint32_t sg = fsign[f];
    for (int k = 0; k < 3; ++k) {
        const float sd = sumd[3 * f + k];
        tz[k] = tw[k] >= 0 ? zin[tw[k]] : zo[k];
        S[k] = tw[k] >= 0 ? sd : 2.f * sd;
        q[k] = (sg >> k) & 1 ? 1.f : -1.f;
    }
    edge_face_update(zo, tz, S, q, c, rmu, mu_relax, zn);
    for (int k = 0; k < 3; ++k) zout[3 * f + k] = zn[k];
}

__global__ void __launch_bounds__(kBlockA) k_admm_edge(int nf, const int32_t* __restrict__ twin,
                                                       const uint8_t* __restrict__ fsign,
                                                       const float* __restrict__ sumd,
                                                       const float* __restrict__ zin, float* __restrict__ zout,
                                                       float rmu, float c, float mu_relax) {
    int f = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    admm_edge_face(f, twin, fsign, sumd, zin, zout, rmu, c, mu_relax);
}

// `iters` iterations per launch over LDS-resident regions (face tiles with
// halos of `iters` rings, see admm_tiles.cpp): one workgroup per tile loads
// its region's copies, target sums and records into LDS and registers, runs
// the iterations (each computes every face's new copies from LDS into
// registers, then after a barrier stores them back: one LDS buffer), and
// writes back its own faces (and, with zprev, their state one iteration
// before the last).  Every face update is the one of
// k_admm_edge, so the result is that of `iters` plain launches.  A halo face
// whose twin lies outside the region uses its own copy in its place; such
// faces are at the region's edge and, like every face d rings out, are
// exact only for iters - d iterations, which the tile's faces never read
// beyond.
// (8 waves per SIMD: two 1024-thread workgroups per CU, so at most 64 VGPRs)
constexpr int kBlockT = 1024;
template <int PER>
__global__ void __launch_bounds__(kBlockT, 8) k_admm_edge_tiled(
    const int32_t* __restrict__ f0, const int32_t* __restrict__ rptr, const int32_t* __restrict__ halo,
    const uint64_t* __restrict__ rec, const float* __restrict__ sumd, const float* __restrict__ zin,
    float* __restrict__ zout, float* __restrict__ zprev, int iters, float rmu, float c, float mu_relax,
    const uint8_t* __restrict__ tile_on) {
    extern __shared__ float zl[];   // 3 copies per region face
    const int p = xcd_block(blockIdx.x, gridDim.x);
    if (tile_on && !tile_on[p]) return;   // a stopped component (the same for the whole workgroup)
    const int a = f0[p], nint = f0[p + 1] - a;
    const int rb = rptr[p], nreg = rptr[p + 1] - rb;
    if (nint == 0) return;   // the same for the whole workgroup
    const int hb = rb - a;
    const int tid = threadIdx.x;
    float* cur = zl;
    // per region face: LDS index of each twin copy (the face's own copy on
    // the boundary and for a twin outside the region), target sums (doubled
    // on the boundary) and signs, kept in registers for the launch
    // (all of a thread's loads are issued before any is used, in two
    // rounds: the halo faces' ids, then the faces' data; threads past the
    // region load the region's last face and discard it)
    int ta[PER][3], g[PER];
    float S[PER][3], q[PER][3], z[PER][3];
    uint64_t R[PER];
    const int nh = nreg - nint;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int r = min(tid + j * kBlockT, nreg - 1);
        g[j] = a + r;
        if (nh > 0) {   // the same for the whole workgroup
            const int hg = halo[hb + min(max(r - nint, 0), nh - 1)];
            if (r >= nint) g[j] = hg;
        }
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int r = min(tid + j * kBlockT, nreg - 1);
        R[j] = rec[rb + r];
        for (int k = 0; k < 3; ++k) {
            S[j][k] = sumd[3 * g[j] + k];
            z[j][k] = zin[3 * g[j] + k];
        }
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int r = tid + j * kBlockT;
        const uint32_t sg = (uint32_t)(R[j] >> 48);
        for (int k = 0; k < 3; ++k) {
            const uint32_t code = (uint32_t)(R[j] >> (16 * k)) & 0xFFFFu;
            ta[j][k] = code >= kTwinOut ? 3 * r + k : (int)code;
            if (code == kTwinNone) S[j][k] = 2.f * S[j][k];
            q[j][k] = (sg >> k) & 1 ? 1.f : -1.f;
        }
        if (r < nreg)
            for (int k = 0; k < 3; ++k) cur[3 * r + k] = z[j][k];
    }
    __syncthreads();
    for (int it = 0; it < iters; ++it) {
        float zn[PER][3];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int r = tid + j * kBlockT;
            if (r >= nreg) continue;
            float zo[3], tz[3];
            for (int k = 0; k < 3; ++k) zo[k] = cur[3 * r + k];
            for (int k = 0; k < 3; ++k) tz[k] = cur[ta[j][k]];
            edge_face_update(zo, tz, S[j], q[j], c, rmu, mu_relax, zn[j]);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int r = tid + j * kBlockT;
            if (r >= nreg) continue;
            for (int k = 0; k < 3; ++k) cur[3 * r + k] = zn[j][k];
        }
        __syncthreads();
        if (zprev && it == iters - 2) {
            for (int r = tid; r < nint; r += kBlockT)
                for (int k = 0; k < 3; ++k) zprev[3 * (a + r) + k] = cur[3 * r + k];
        }
    }
    for (int r = tid; r < nint; r += kBlockT)
        for (int k = 0; k < 3; ++k) zout[3 * (a + r) + k] = cur[3 * r + k];
}

// A component that stops (cflag 1): its faces' state copied into the other
// buffer and the one-iteration-back buffer, so that launches that skip its
// tiles leave it in place; tile_on follows the flags.
__global__ void k_freeze_faces(int nf, const int32_t* __restrict__ tri, const int32_t* __restrict__ comp,
                               const uint8_t* __restrict__ cflag, const float* __restrict__ za, float* zb,
                               float* zback) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf || cflag[comp[tri[3 * f]]] != 1) return;
    for (int k = 0; k < 3; ++k) {
        zb[3 * f + k] = za[3 * f + k];
        zback[3 * f + k] = za[3 * f + k];
    }
}
__global__ void k_tiles_on(int nt, const int32_t* __restrict__ tile_comp, const uint8_t* __restrict__ cflag,
                           uint8_t* tile_on) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nt) tile_on[p] = cflag ? (uint8_t)(cflag[tile_comp[p]] == 0) : (uint8_t)1;
}

// r_p = w' - x' with w' = x + (zeta' - zeta)/(mu alpha) (from the zeta
// update), r_d = mu (x' - x).  partial = (sum r_p^2, sum r_d^2) per block.
__global__ void k_resid_edge(int nf, const int32_t* twin, const float* sumz, const float* za, const float* zb,
                             float mu, float inv1mu, float mu_relax, double* partial) {
    int f = blockIdx.x * blockDim.x + threadIdx.x;
    double rp = 0.0, rd = 0.0;
    if (f < nf) {
        for (int k = 0; k < 3; ++k) {
            const int h = 3 * f + k, t = twin[h];
            const int bnd = t < 0;
            float xa = edge_x(sumz[h], za[h], bnd ? 0.f : za[t], bnd, inv1mu);
            float xb = edge_x(sumz[h], zb[h], bnd ? 0.f : zb[t], bnd, inv1mu);
            double wn = (double)xa + ((double)zb[h] - (double)za[h]) / mu_relax;
            double p = wn - (double)xb;
            double d = (double)mu * ((double)xb - (double)xa);
            rp += p * p;
            rd += d * d;
        }
    }
    rp = block_sum2(rp);
    rd = block_sum2(rd);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = rp;
        partial[2 * blockIdx.x + 1] = rd;
    }
}

__global__ void k_reduce_pairs(double* partial, int n) {
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        a += partial[2 * i];
        b += partial[2 * i + 1];
    }
    a = block_sum2(a);
    b = block_sum2(b);
    if (threadIdx.x == 0) {
        partial[2 * n] = a;
        partial[2 * n + 1] = b;
    }
}

__global__ void k_edge_x(int ne, const int32_t* h01, const int32_t* ef, const float* sumz, const float* z,
                         float inv1mu, float* x) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    int bnd = ef[2 * e + 1] < 0;
    const int h0 = h01[2 * e], h1 = h01[2 * e + 1];
    x[e] = edge_x(sumz[e], z[h0], h1 >= 0 ? z[h1] : 0.f, bnd, inv1mu);
}

// ------------------------------------------------- source paths (Eqs. 24-25)
// Each path S of w.paths (a source path, or a generator loop of Sec. 5.1)
// adds a group of copies with the constraint of Eq. 25 / 23 (edge form) or
// Eq. 24 / 22 (face form); their duals are folded like the face copies.
// In both forms one launch holds the face update and the chunk sums of
// every group's projection (chunks of kPathChunk slots, from the state the
// face kernel reads), then k_path_*_fix (one thread per edge or face
// carrying copies) projects the copies with their group's sums and
// completes the update the face kernel did without them.
//
// Edge form.  Per path slot keep zeta_S = kappa + mu v_hat; with n_e path
// slots on edge e the X-update becomes
//   x_e = (S_e + sum_faces zeta + sum_slots zeta_S) / (|H_e| (1 + mu) + mu n_e).
// The face kernel keeps its formula x_e = (S'_e + sum_faces zeta) / (|H_e| (1 + mu))
// on an effective target sum S'_e = x_e |H_e| (1 + mu) - sum_faces zeta, which
// the fix kernel writes for path edges (in FP64: both terms are ~mu^2 times
// larger than their difference).  The projection of a path's copies is
//   t = 2 x - zeta_S / mu,  v = t - (s.t / |S|) s,  zeta_S' = zeta_S + mu alpha (v - x).
//
// Face form.  Per path slot keep z_S = y_S + kappa / (mu alpha_f) for the face
// f chosen on the slot's edge; q = 2 g_f - z_S, the weighted projection onto
// sum_j e_j . y_j = 0 is y_j = q_j - (c / A_j) e_j with
// c = sum_j e_j . q_j / sum_j |e_j|^2 / A_j, z_S' = z_S + alpha (y - g_f), and the
// fix kernel redoes the G-update of a face with its path copies included.

__device__ inline double block_sum_all(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
    return r;
}

__global__ void k_path_edge_zinit(int ns, const int32_t* edge, const int32_t* ef, const float* sumz, float mu,
                                  float* zp) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ns) return;
    int e = edge[k];
    float nh = ef[2 * e + 1] >= 0 ? 2.f : 1.f;
    zp[k] = mu * (sumz[e] / nh);   // kappa = 0, v = x = mean target
}

// Edge-form projection, first half: chunk c of path p sums s . t over its
// slots (t = 2 x - zeta_S / mu with x from the previous state), one
// workgroup per chunk of kPathChunk slots; pc[c] = the chunk's sum.
__device__ inline void path_edge_chunk_block(int c, const int32_t* __restrict__ chunk_path,
                                             const int32_t* __restrict__ cptr, const int32_t* __restrict__ ptr,
                                             const int32_t* __restrict__ edge, const float* __restrict__ sign,
                                             const int2* __restrict__ zslot, const float* __restrict__ seff,
                                             const float* __restrict__ zin, const float* __restrict__ zp,
                                             double* __restrict__ pc, float mu, float inv1mu, double* sh) {
    const int p = chunk_path[c];
    const int b = ptr[p] + (c - cptr[p]) * kPathChunk;
    const int end = min(ptr[p + 1], b + kPathChunk);
    double acc = 0.0;
    for (int k = b + threadIdx.x; k < end; k += blockDim.x) {
        const int e = edge[k];
        const int2 hh = zslot[k];
        const float x = edge_x(seff[e], zin[hh.x], hh.y >= 0 ? zin[hh.y] : 0.f, hh.y < 0, inv1mu);
        acc += (double)sign[k] * (double)(2.f * x - zp[k] / mu);
    }
    acc = block_sum_all(acc, sh);
    if (threadIdx.x == 0) pc[c] = acc;
}

// The face update and the chunk sums of one iteration in one launch: blocks
// [0, nch) sum one chunk each, blocks [nch, nch + nfb) update faces (both
// read the previous state only and write disjoint outputs).
__global__ void __launch_bounds__(kBlockA) k_admm_edge_paths(
    int nf, int nfb, int nch, const int32_t* __restrict__ twin, const uint8_t* __restrict__ fsign,
    const float* __restrict__ sumd, const float* __restrict__ zin, float* __restrict__ zout,
    const int32_t* __restrict__ chunk_path, const int32_t* __restrict__ cptr, const int32_t* __restrict__ ptr,
    const int32_t* __restrict__ edge, const float* __restrict__ sign, const int2* __restrict__ zslot,
    const float* __restrict__ seff, const float* __restrict__ zp, double* __restrict__ pc, float mu, float rmu,
    float inv1mu, float mu_relax) {
    __shared__ double sh[kBlockA / 64];
    if ((int)blockIdx.x < nch) {
        path_edge_chunk_block((int)blockIdx.x, chunk_path, cptr, ptr, edge, sign, zslot, seff, zin, zp, pc, mu,
                              inv1mu, sh);
        return;
    }
    const int f = xcd_block((int)blockIdx.x - nch, nfb) * blockDim.x + threadIdx.x;
    if (f < nf) admm_edge_face(f, twin, fsign, sumd, zin, zout, rmu, 0.5f * inv1mu, mu_relax);
}

// Second half, one thread per edge carrying path slots: each slot's copy is
// projected with its path's mean c = (sum of the path's chunk sums) / |S|,
//   v = t - c s,  zeta_S' = zeta_S + mu alpha (v - x),
// then the edge's X-update with those copies included gives the effective
// target sum S' that the face kernel reads next (FP64: both terms are ~mu^2
// times larger than their difference).
__global__ void k_path_edge_fix(int ng, const int32_t* gptr, const int32_t* gid, const int32_t* gslot,
                                const int32_t* spath, const int32_t* ptr, const int32_t* cptr, const double* pc,
                                const float* sign, float* zp, const float* sumz, const float* zin, const float* zout,
                                const int2* gzslot, float muf, float inv1mu, float mu_relax, float* seff,
                                float* sumd) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    const int e = gid[g];
    const int h0 = gzslot[g].x, h1 = gzslot[g].y;
    const bool bnd = h1 < 0;
    const float xo = edge_x(seff[e], zin[h0], bnd ? 0.f : zin[h1], bnd, inv1mu);
    double P = 0.0;
    for (int j = gptr[g]; j < gptr[g + 1]; ++j) {
        const int k = gslot[j];
        const int p = spath[k];
        double sum = 0.0;
        for (int c = cptr[p]; c < cptr[p + 1]; ++c) sum += pc[c];
        const float cc = (float)(sum / (double)(ptr[p + 1] - ptr[p]));
        const float z = zp[k];
        const float t = 2.f * xo - z / muf;
        const float v = t - cc * sign[k];
        const float zn = z + mu_relax * (v - xo);
        zp[k] = zn;
        P += zn;
    }
    const int n = gptr[g + 1] - gptr[g];
    const double mu = muf;
    const double Z = (double)zout[h0] + (bnd ? 0.0 : (double)zout[h1]);
    const double D0 = (bnd ? 1.0 : 2.0) * (1.0 + mu);
    const double x = ((double)sumz[e] + P + Z) / (D0 + mu * n);
    const float sp = (float)(x * D0 - Z);
    seff[e] = sp;
    sumd[h0] = sp;   // the face kernel reads S' per slot
    if (!bnd) sumd[h1] = sp;
}

__global__ void k_path_face_zinit(int ns, const int32_t* face, const float* h, float* zp) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ns) return;
    int f = face[k];
    for (int c = 0; c < 3; ++c) zp[3 * k + c] = h[3 * f + c];   // y = g = h, kappa = 0
}

// Second half, one thread per face carrying group copies: each copy is
// projected with its group's c = (sum e.q) / (sum |e|^2 / A):
//   y = q - (c / A_f) e,  z_S' = z_S + alpha (y - g_f),
// then the face's G-update is redone with those copies included.
__global__ void k_path_face_fix(int ng, const int32_t* gptr, const int32_t* gid, const int32_t* gslot,
                                const int32_t* spath, const int32_t* cptr, const double* pc, const float* vec,
                                const double* farea, const float* gin, float* zp, const uint32_t* fslot,
                                const float* zout, const float* h, float mu, float relax, float* gout) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    const int f = gid[g];
    const float go[3] = {gin[3 * f], gin[3 * f + 1], gin[3 * f + 2]};
    float acc[3] = {0.f, 0.f, 0.f};
    int cnt = 0;
    for (int k = 0; k < 3; ++k) {
        uint32_t sl = fslot[3 * f + k];
        if (slot_bnd(sl)) continue;
        const float* z = zout + 9 * f + 3 * k;
        for (int c = 0; c < 3; ++c) acc[c] += z[c];
        ++cnt;
    }
    for (int j = gptr[g]; j < gptr[g + 1]; ++j) {
        const int k = gslot[j];
        const int p = spath[k];
        double dot = 0.0, den = 0.0;
        for (int c = cptr[p]; c < cptr[p + 1]; ++c) {
            dot += pc[2 * c];
            den += pc[2 * c + 1];
        }
        const float ca = (float)(dot / den / farea[f]);
        float* z = zp + 3 * k;
        for (int c = 0; c < 3; ++c) {
            const float q = 2.f * go[c] - z[c];
            const float y = q - ca * vec[3 * k + c];
            const float zn = z[c] + relax * (y - go[c]);
            z[c] = zn;
            acc[c] += zn;
        }
        ++cnt;
    }
    const float dn = 1.f / (2.f + mu * (float)cnt);
    for (int c = 0; c < 3; ++c) gout[3 * f + c] = (2.f * h[3 * f + c] + mu * acc[c]) * dn;
}

static void reduce_pair(Mesh& m, Work& w, int nblocks, hipStream_t s, double& a, double& b) {
    hipLaunchKernelGGL(k_reduce_pairs, dim3(1), dim3(kBlockA), 0, s, w.partial.p, nblocks);
    HG_CHECK_HIP(hipGetLastError());
    HG_CHECK_HIP(
        hipMemcpyAsync(w.pinned, w.partial.p + 2 * nblocks, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HG_CHECK_HIP(hipStreamSynchronize(s));
    a = w.pinned[0];
    b = w.pinned[1];
}

AdmmResult run_admm_edge(Mesh& m, Work& w, int iters, const hg_opts& o, hipStream_t s, int depth, bool use_paths) {
    const int nf = (int)m.nf, ne = (int)m.ne;
    w.sumz.alloc(ne);
    w.z0.alloc((size_t)3 * nf);
    w.z1.alloc((size_t)3 * nf);
    w.sumd.alloc((size_t)3 * nf);
    w.xe.alloc(ne);
    const float mu = (float)o.mu, inv1mu = 1.0f / (1.0f + mu), mu_relax = (float)(o.mu * o.relax);
    const float rmu = 1.0f / mu, chalf = 0.5f * inv1mu;
    const int gf = grid_for(nf, kBlockA), ge = grid_for(ne, kBlockA);
    if ((int)w.partial.n < 2 * gf + 8) w.partial.alloc((size_t)2 * gf + 8);
    if (m.intrinsic)
        hipLaunchKernelGGL(k_edge_targets_local, dim3(ge), dim3(kBlockA), 0, s, ne, m.ef.p, m.fslot.p, m.fsign.p,
                           m.floc.p, w.h.p, w.sumz.p);
    else
        hipLaunchKernelGGL(k_edge_targets, dim3(ge), dim3(kBlockA), 0, s, ne, m.ev.p, m.ef.p, m.px.p, m.py.p,
                           m.pz.p, w.h.p, w.sumz.p);
    hipLaunchKernelGGL(k_zeta_init, dim3(ge), dim3(kBlockA), 0, s, ne, m.h01.p, w.sumz.p, mu, w.z0.p, w.sumd.p);
    HG_CHECK_HIP(hipGetLastError());
    auto& P = w.paths;
    use_paths = use_paths && P.np > 0;
    const float* S = w.sumz.p;   // target sums as the face kernel sees them
    if (use_paths) {
        P.z.alloc(P.ns);
        P.seff.alloc(ne);
        HG_CHECK_HIP(hipMemcpyAsync(P.seff.p, w.sumz.p, (size_t)ne * sizeof(float), hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_path_edge_zinit, dim3(grid_for(P.ns, kBlockA)), dim3(kBlockA), 0, s, P.ns, P.edge.p,
                           m.ef.p, w.sumz.p, mu, P.z.p);
        HG_CHECK_HIP(hipGetLastError());
        S = P.seff.p;
    }
    AdmmResult r;
    const bool fixed = iters > 0;
    const bool monitor = !fixed && depth >= 0;
    const int cap = fixed ? iters : o.max_admm;
    // blocked launches (several iterations each) without constraint groups:
    // the largest block size up to the requested one whose regions fit
    const Mesh::EdgeTileSet* tiles = nullptr;
    int K = 1;
    // requested block: the option, else the mesh's autotuned one, else 6
    const int req = o.admm_block > 0 ? o.admm_block : (m.tuned_admm_block > 0 ? m.tuned_admm_block : kAutoAdmmBlock);
    for (int k = use_paths ? 1 : req; k > 1 && !tiles; --k)
        if ((tiles = m.ensure_edge_tiles(k, s))) K = k;
    const int per = tiles ? (tiles->max_region + kBlockT - 1) / kBlockT : 0;
    r.block = K;
    // Several connected components (meshes joined into one batch): each
    // keeps its own check schedule (a check covers only the components due
    // for one) and stops on its own distance check, as it would alone; its
    // tiles then sit out the remaining launches (its state is copied into
    // both buffers first, so the skipped launches leave it in place).  A
    // face tile's component is its vertex tile's.
    const int ncomp = std::max(1, m.n_comp);
    const bool percomp =
        monitor && tiles && !use_paths && ncomp > 1 && o.tol_seam <= 0.0 && tiles->n == m.n_patches;
    std::vector<DistStop> cstop;
    std::vector<uint8_t> cflag_h, cdue_h;
    std::vector<int> cnext, cint;   // per component: its next check, iterations between checks
    if (percomp) {
        w.tile_on.alloc((size_t)tiles->n);
        w.cflag.alloc((size_t)ncomp);
        hipLaunchKernelGGL(k_tiles_on, dim3(grid_for(tiles->n, kBlockA)), dim3(kBlockA), 0, s, tiles->n,
                           m.tile_comp.p, nullptr, w.tile_on.p);
        HG_CHECK_HIP(hipGetLastError());
        cstop.assign((size_t)ncomp, DistStop());
        cflag_h.assign((size_t)ncomp, 0);
        cdue_h.assign((size_t)ncomp, 0);
    }
    const uint8_t* tile_on = percomp ? w.tile_on.p : nullptr;
    const int check = monitor ? std::max(64, o.check_every) : std::max(1, o.check_every);
    // iterations between two checks: one chunk, or kCoarseChecks chunks far
    // from convergence (DistStop)
    int interval = check, next_check = check;
    if (percomp) {
        cnext.assign((size_t)ncomp, check);
        cint.assign((size_t)ncomp, check);
    }
    float* za = w.z0.p;
    float* zb = w.z1.p;
    // algorithmic bytes of one launch: per face its three zeta, S copies
    // and twin slots and its sign byte read, its three zeta written (the
    // twins' zeta are the same array, read by their own faces); blocked:
    // per face its record, three zeta and S copies read and three zeta
    // written once (halo re-reads and the occasional extra write of the
    // state one iteration back are overhead)
    r.bytes_per_iter = (uint64_t)(tiles ? 44 : 49) * nf;
    // path kernels: chunk sums read per slot its edge, slot pair, S', zeta
    // pair, sign and copy (28 B) and write 8 B per chunk; the fix reads per
    // slot its index, path, sign and copy and writes the copy (20 B), per
    // group its slot range, id, slot pair, S', old and new zeta pairs and S
    // and writes S' three times (52 B)
    if (use_paths)
        r.bytes_per_iter += (uint64_t)48 * P.ns + (uint64_t)8 * P.nch + (uint64_t)52 * P.ng_edge;
    RunTimer rt;
    int run_len = 0;
    DistStop stop;
    // residuals as rms over the 3|F| copies, r_p / hbar and r_d / (mu hbar)
    auto residuals = [&](const float* prev, const float* cur) {
        hipLaunchKernelGGL(k_resid_edge, dim3(gf), dim3(kBlockA), 0, s, nf, m.twin.p, w.sumd.p, prev, cur, mu,
                           inv1mu, mu_relax, w.partial.p);
        double a, b;
        reduce_pair(m, w, gf, s, a, b);
        r.rp = sqrt(a) / (sqrt(3.0 * (double)nf) * m.hbar);
        r.rd = sqrt(b) / (sqrt(3.0 * (double)nf) * m.hbar * o.mu);
    };
    // one iteration from state zi into zo (the face kernel, then the path
    // constraint groups)
    auto iterate = [&](float* zi, float* zo) {
        if (!use_paths) {
            hipLaunchKernelGGL(k_admm_edge, dim3(gf), dim3(kBlockA), 0, s, nf, m.twin.p, m.fsign.p, w.sumd.p, zi, zo,
                               rmu, chalf, mu_relax);
        } else {
            hipLaunchKernelGGL(k_admm_edge_paths, dim3(gf + P.nch), dim3(kBlockA), 0, s, nf, gf, P.nch, m.twin.p,
                               m.fsign.p, w.sumd.p, zi, zo, P.chunk_path.p, P.cptr.p, P.ptr.p, P.edge.p, P.sign.p,
                               P.zslot.p, S, P.z.p, P.pc.p, mu, rmu, inv1mu, mu_relax);
            hipLaunchKernelGGL(k_path_edge_fix, dim3(grid_for(P.ng_edge, kBlockA)), dim3(kBlockA), 0, s, P.ng_edge,
                               P.eg_ptr.p, P.eg_id.p, P.eg_slot.p, P.spath.p, P.ptr.p, P.cptr.p, P.pc.p, P.sign.p,
                               P.z.p, w.sumz.p, zi, zo, P.gzslot.p, mu, inv1mu, mu_relax, P.seff.p, w.sumd.p);
        }
    };
    // n <= K iterations from zi into zo in one launch (the regions' K-ring
    // halos cover any n up to K); with zp, zp also receives the state one
    // iteration before zo's
    auto iterate_block = [&](float* zi, float* zo, float* zp, int n) {
        const size_t lds = (size_t)3 * tiles->max_region * sizeof(float);
        switch (per) {
#define HG_TILED(P)                                                                                              \
    case P:                                                                                                      \
        hipLaunchKernelGGL(k_admm_edge_tiled<P>, dim3(tiles->n), dim3(kBlockT), lds, s, tiles->f0.p,             \
                           tiles->rptr.p, tiles->halo.p, tiles->rec.p, w.sumd.p, zi, zo, zp, n, rmu, chalf,        \
                           mu_relax, tile_on);                                                                   \
        break;
            HG_TILED(1)
            HG_TILED(2)
            HG_TILED(3)
            HG_TILED(4)
#undef HG_TILED
            default: throw Error{HG_E_DEVICE, "blocked ADMM: region too large"};
        }
    };
    // a run of n iterations from za: blocked launches of K, then one of the
    // remaining iterations (a single iteration runs the plain kernel); the
    // last blocked launch also keeps the state one iteration back (in w.h,
    // whose directions the edge form has already turned into targets).
    // Returns the launches and sets prev to the state one iteration before
    // a's.  (With enqueue = false only the buffer roles are followed, for a
    // run replayed from a graph.)
    float* zback = w.h.p;
    const float* zprev = zb;
    auto run = [&](int n, float*& a, float*& b, const float*& prev, bool enqueue) {
        const int nb = tiles ? n / K : 0;
        const int rest = n - nb * K;
        const bool tail = tiles && rest >= 2;   // the remainder as one blocked launch
        const int nl = nb + (tail ? 1 : 0);
        const int single = tail ? 0 : rest;
        for (int k = 0; k < nl; ++k) {
            const int it_k = k < nb ? K : rest;
            if (enqueue) iterate_block(a, b, (k == nl - 1 && single == 0) ? zback : nullptr, it_k);
            std::swap(a, b);
        }
        for (int k = 0; k < single; ++k) {
            if (enqueue) iterate(a, b);
            std::swap(a, b);   // a is now the current state, b the previous
        }
        prev = single > 0 || nl == 0 ? b : zback;
        return nl + single;
    };
    // runs of `check` iterations between two checks, one captured graph per
    // starting buffer (a run may swap the buffers' roles)
    GraphChunk graph[2];
    const bool graphs = !fixed && o.use_graphs;
    int it = 0;
    while (it < cap) {
        const int n = std::min(check - it % check, cap - it);
        GraphChunk& gr = graph[za == w.z0.p ? 0 : 1];
        rt.start(s);
        int launches = 0;
        if (graphs && n == check && !gr.tried) {
            float *a = za, *b = zb;
            const float* pv = nullptr;
            gr.capture(s, [&] { (void)run(n, a, b, pv, true); });
        }
        if (graphs && n == check && gr.ready()) {
            gr.launch(s);
            launches = run(n, za, zb, zprev, false);
        } else {
            launches = run(n, za, zb, zprev, true);
        }
        HG_CHECK_HIP(hipGetLastError());
        it += n;
        r.iters = it;
        r.launches += launches;
        run_len = launches;
        r.kernel_ms += rt.stop(s);
        r.timed_launches += run_len;
        bool want = it >= next_check || it == cap;
        if (percomp) {   // the components still iterating whose check is due
            want = false;
            for (int c = 0; c < ncomp; ++c) {
                cdue_h[c] = cflag_h[c] == 0 && (it >= cnext[c] || it == cap) ? 1 : 0;
                want = want || cdue_h[c] != 0;
            }
        }
        if (!fixed && want) {
            bool done;
            const EdgeX ex{S, za, inv1mu};
            if (percomp) {
                std::vector<double> dl, dm;
                dist_change_comp(m, w, HG_FORM_EDGE, depth, nullptr, nullptr, stop.first, s, dl, dm, &ex,
                                 cdue_h.data());
                stop.first = false;
                bool stopping = false;
                for (int c = 0; c < ncomp; ++c) {
                    if (cflag_h[c] != 0) {   // stopped at an earlier check
                        cflag_h[c] = 2;
                        continue;
                    }
                    if (!cdue_h[c]) continue;
                    // the schedule of a solve alone (below): checks every
                    // chunk, or every kCoarseChecks chunks while far
                    DistStop& cs = cstop[c];
                    if (cs.update(dl[c], dm[c], o.tol_admm)) {
                        cflag_h[c] = 1;
                        stopping = true;
                        continue;
                    }
                    if (cint[c] == check && cs.far(dm[c], o.tol_admm)) {
                        cint[c] = kCoarseChecks * check;
                        cs.restart();
                    } else if (cint[c] > check && cs.near(dm[c], o.tol_admm)) {
                        cint[c] = check;
                        cs.restart();
                    }
                    cnext[c] = it + cint[c];
                }
                done = true;
                for (int c = 0; c < ncomp && done; ++c) done = cflag_h[c] != 0;
                if (!done && stopping) {
                    HG_CHECK_HIP(hipMemcpyAsync(w.cflag.p, cflag_h.data(), (size_t)ncomp, hipMemcpyHostToDevice, s));
                    hipLaunchKernelGGL(k_freeze_faces, dim3(gf), dim3(kBlockA), 0, s, nf, m.tri.p, m.comp_v.p,
                                       w.cflag.p, za, zb, zback);
                    hipLaunchKernelGGL(k_tiles_on, dim3(grid_for(tiles->n, kBlockA)), dim3(kBlockA), 0, s,
                                       tiles->n, m.tile_comp.p, w.cflag.p, w.tile_on.p);
                    HG_CHECK_HIP(hipGetLastError());
                    // cflag_h is read by the copy before the next check rewrites it
                    HG_CHECK_HIP(hipStreamSynchronize(s));
                }
            } else if (monitor) {
                // the change needs x only on the edges the integration follows
                double delta, dmax;
                dist_change(m, w, HG_FORM_EDGE, depth, nullptr, nullptr, stop.first, s, delta, dmax, nullptr, &ex);
                done = stop.update(delta, dmax, o.tol_admm);
                // the seam (x on every edge) only once the distance has settled
                if (done && o.tol_seam > 0.0) {
                    hipLaunchKernelGGL(k_edge_x, dim3(ge), dim3(kBlockA), 0, s, ne, m.h01.p, m.ef.p, S, za, inv1mu,
                                       w.xe.p);
                    r.seam = seam_now(m, w, HG_FORM_EDGE, w.xe.p, nullptr, s) / m.hbar;
                    done = r.seam <= o.tol_seam;
                }
                if (!done && interval == check && stop.far(dmax, o.tol_admm)) {
                    interval = kCoarseChecks * check;
                    stop.restart();
                } else if (!done && interval > check && stop.near(dmax, o.tol_admm)) {
                    interval = check;
                    stop.restart();
                }
            } else {
                residuals(zprev, za);
                done = r.rp <= o.tol_admm && r.rd <= o.tol_admm;
            }
            next_check = it + interval;
            if (done) {
                r.converged = true;
                break;
            }
        }
    }
    if (rt.open) {
        r.kernel_ms += rt.stop(s);
        r.timed_launches += run_len;
    }
    if (fixed) r.converged = true;
    if (r.iters > 0) residuals(zprev, za);
    hipLaunchKernelGGL(k_edge_x, dim3(ge), dim3(kBlockA), 0, s, ne, m.h01.p, m.ef.p, S, za, inv1mu, w.xe.p);
    HG_CHECK_HIP(hipGetLastError());
    // the seam of the final state (its d is the last check's), once
    if (monitor && !stop.first && o.tol_seam <= 0.0)
        r.seam = seam_now(m, w, HG_FORM_EDGE, w.xe.p, nullptr, s) / m.hbar;
    if (za != w.z0.p)
        HG_CHECK_HIP(hipMemcpyAsync(w.z0.p, za, (size_t)3 * nf * sizeof(float), hipMemcpyDeviceToDevice, s));
    return r;
}

// ---------------------------------------------------------------- face form
// z layout: slot-major, the copy of face f on its slot k at z[3 (3f + k)];
// every copy starts at h_f (a boundary slot's copy is never read).
__global__ void k_face_init(int nf, const float* h, float* g, float* z) {
    int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    for (int d = 0; d < 3; ++d) {
        const float v = h[3 * f + d];
        g[3 * f + d] = v;
        z[9 * f + d] = v;
        z[9 * f + 3 + d] = v;
        z[9 * f + 6 + d] = v;
    }
}

// One face's Y/Z/G update.  Per slot k with a neighbour (twin slot t, face
// t / 3): the two copies' W-projection onto the compatibility of Eq. 10 is
// y_own = q_own + w (e . (q_nb - q_own)) e with q = 2 g - z, e the unit edge
// vector and w = A_nb / (A_own + A_nb) (sgeo[slot] = (e, w)); then
// z' = z + alpha (y - g) and g' = (2 h + mu sum z') / (2 + mu n).
__device__ inline void admm_face_one(int f, const int32_t* __restrict__ twin, const float4* __restrict__ sgeo,
                                     const float* __restrict__ h, const float* __restrict__ gin,
                                     const float* __restrict__ zin, float* __restrict__ gout,
                                     float* __restrict__ zout, float mu, float relax) {
    const float g0 = gin[3 * f], g1 = gin[3 * f + 1], g2 = gin[3 * f + 2];
    int tw[3];
    float zo[9];
    for (int k = 0; k < 3; ++k) tw[k] = twin[3 * f + k];
    for (int i = 0; i < 9; ++i) zo[i] = zin[9 * f + i];
    float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f;
    int cnt = 0;
    for (int k = 0; k < 3; ++k) {
        const int t = tw[k];
        if (t < 0) continue;
        const int nb = t / 3;
        const float4 sg = sgeo[3 * f + k];
        const float* zn = zin + 3 * t;
        float qo0 = 2.f * g0 - zo[3 * k], qo1 = 2.f * g1 - zo[3 * k + 1], qo2 = 2.f * g2 - zo[3 * k + 2];
        float qn0 = 2.f * gin[3 * nb] - zn[0];
        float qn1 = 2.f * gin[3 * nb + 1] - zn[1];
        float qn2 = 2.f * gin[3 * nb + 2] - zn[2];
        float sdot = sg.x * (qn0 - qo0) + sg.y * (qn1 - qo1) + sg.z * (qn2 - qo2);
        float c = sg.w * sdot;
        float z0n = zo[3 * k] + relax * (qo0 + c * sg.x - g0);
        float z1n = zo[3 * k + 1] + relax * (qo1 + c * sg.y - g1);
        float z2n = zo[3 * k + 2] + relax * (qo2 + c * sg.z - g2);
        float* zw = zout + 9 * f + 3 * k;
        zw[0] = z0n;
        zw[1] = z1n;
        zw[2] = z2n;
        acc0 += z0n;
        acc1 += z1n;
        acc2 += z2n;
        ++cnt;
    }
    const float den = 1.f / (2.f + mu * (float)cnt);
    gout[3 * f] = (2.f * h[3 * f] + mu * acc0) * den;
    gout[3 * f + 1] = (2.f * h[3 * f + 1] + mu * acc1) * den;
    gout[3 * f + 2] = (2.f * h[3 * f + 2] + mu * acc2) * den;
}

__global__ void __launch_bounds__(kBlockA) k_admm_face(int nf, const int32_t* __restrict__ twin,
                                                       const float4* __restrict__ sgeo,
                                                       const float* __restrict__ h, const float* __restrict__ gin,
                                                       const float* __restrict__ zin, float* __restrict__ gout,
                                                       float* __restrict__ zout, float mu, float relax) {
    int f = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    admm_face_one(f, twin, sgeo, h, gin, zin, gout, zout, mu, relax);
}

// Face-form projection of the constraint groups, first half: chunk c of
// group p sums e_j . (2 g_f - z_j) and |e_j|^2 / A_f over its slots (from
// the state the face kernel reads); pc[2c], pc[2c+1] = the two sums.
__device__ inline void path_face_chunk_block(int c, const int32_t* __restrict__ chunk_path,
                                             const int32_t* __restrict__ cptr, const int32_t* __restrict__ ptr,
                                             const int32_t* __restrict__ face, const float* __restrict__ vec,
                                             const double* __restrict__ farea, const float* __restrict__ gin,
                                             const float* __restrict__ zp, double* __restrict__ pc, double* sh) {
    const int p = chunk_path[c];
    const int b = ptr[p] + (c - cptr[p]) * kPathChunk;
    const int end = min(ptr[p + 1], b + kPathChunk);
    double dot = 0.0, den = 0.0;
    for (int k = b + threadIdx.x; k < end; k += blockDim.x) {
        const int f = face[k];
        double ee = 0.0;
        for (int q = 0; q < 3; ++q) {
            const double ec = vec[3 * k + q];
            dot += ec * (double)(2.f * gin[3 * f + q] - zp[3 * k + q]);
            ee += ec * ec;
        }
        den += ee / farea[f];
    }
    dot = block_sum_all(dot, sh);
    den = block_sum_all(den, sh);
    if (threadIdx.x == 0) {
        pc[2 * c] = dot;
        pc[2 * c + 1] = den;
    }
}

// The face update and the chunk sums in one launch: blocks [0, nch) sum one
// chunk each, blocks [nch, nch + nfb) update faces.
__global__ void __launch_bounds__(kBlockA) k_admm_face_paths(
    int nf, int nfb, int nch, const int32_t* __restrict__ twin, const float4* __restrict__ sgeo,
    const double* __restrict__ farea, const float* __restrict__ h,
    const float* __restrict__ gin, const float* __restrict__ zin, float* __restrict__ gout, float* __restrict__ zout,
    const int32_t* __restrict__ chunk_path, const int32_t* __restrict__ cptr, const int32_t* __restrict__ ptr,
    const int32_t* __restrict__ face, const float* __restrict__ vec, const float* __restrict__ zp,
    double* __restrict__ pc, float mu, float relax) {
    __shared__ double sh[kBlockA / 64];
    if ((int)blockIdx.x < nch) {
        path_face_chunk_block((int)blockIdx.x, chunk_path, cptr, ptr, face, vec, farea, gin, zp, pc, sh);
        return;
    }
    const int f = xcd_block((int)blockIdx.x - nch, nfb) * blockDim.x + threadIdx.x;
    if (f < nf) admm_face_one(f, twin, sgeo, h, gin, zin, gout, zout, mu, relax);
}

// Per copy k of face i: r_p = sqrt(A_i) (y' - g') with y' = g + (z' - z)/alpha
// (from the z update), r_d = mu A_i (g' - g).
// partial = (sum |r_p|^2, sum |r_d|^2).
__global__ void k_resid_face(int nf, const uint32_t* fslot, const double* farea, const float* ga, const float* gb,
                             const float* za, const float* zb, float mu, float relax, double* partial) {
    int f = blockIdx.x * blockDim.x + threadIdx.x;
    double rp = 0.0, rd = 0.0;
    if (f < nf) {
        double A = farea[f];
        double al = sqrt(A);
        for (int k = 0; k < 3; ++k) {
            uint32_t sl = fslot[3 * f + k];
            if (slot_bnd(sl)) continue;
            const int c = 3 * f + k;   // the copy's slot
            for (int d = 0; d < 3; ++d) {
                double yn = (double)ga[3 * f + d] + ((double)zb[3 * c + d] - (double)za[3 * c + d]) / relax;
                double p = al * (yn - (double)gb[3 * f + d]);
                double q = (double)mu * A * ((double)gb[3 * f + d] - ga[3 * f + d]);
                rp += p * p;
                rd += q * q;
            }
        }
    }
    rp = block_sum2(rp);
    rd = block_sum2(rd);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = rp;
        partial[2 * blockIdx.x + 1] = rd;
    }
}

// |M|_F^2 = sum over copies of the face area
__global__ void k_normM(int nf, const uint32_t* fslot, const double* farea, double* partial) {
    int f = blockIdx.x * blockDim.x + threadIdx.x;
    double a = 0.0;
    if (f < nf)
        for (int k = 0; k < 3; ++k)
            if (!slot_bnd(fslot[3 * f + k])) a += farea[f];
    a = block_sum2(a);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = a;
        partial[2 * blockIdx.x + 1] = 0.0;
    }
}

static void face_residuals(Mesh& m, Work& w, int gf, const float* gprev, const float* gcur, const float* zprev,
                           const float* zcur, float mu, double relax, double normM, hipStream_t s, AdmmResult& r) {
    hipLaunchKernelGGL(k_resid_face, dim3(gf), dim3(kBlockA), 0, s, (int)m.nf, m.fslot.p, m.farea.p, gprev, gcur, zprev,
                       zcur, mu, (float)relax, w.partial.p);
    HG_CHECK_HIP(hipGetLastError());
    double a, b;
    reduce_pair(m, w, gf, s, a, b);
    r.rp = sqrt(a) / normM;
    r.rd = sqrt(b) / normM;
}

AdmmResult run_admm_face(Mesh& m, Work& w, int iters, const hg_opts& o, hipStream_t s, int depth, bool use_paths) {
    const int nf = (int)m.nf, ne = (int)m.ne;
    m.ensure_sgeo(s);
    w.g0.alloc((size_t)3 * nf);
    w.g1.alloc((size_t)3 * nf);
    w.z0.alloc((size_t)9 * nf);
    w.z1.alloc((size_t)9 * nf);
    w.gf.alloc((size_t)3 * nf);
    const float mu = (float)o.mu;
    const int gf = grid_for(nf, kBlockA);
    if ((int)w.partial.n < 2 * gf + 8) w.partial.alloc((size_t)2 * gf + 8);
    hipLaunchKernelGGL(k_face_init, dim3(gf), dim3(kBlockA), 0, s, nf, w.h.p, w.g0.p, w.z0.p);
    auto& P = w.paths;
    use_paths = use_paths && P.np > 0;
    if (use_paths) {
        P.z.alloc((size_t)3 * P.ns);
        hipLaunchKernelGGL(k_path_face_zinit, dim3(grid_for(P.ns, kBlockA)), dim3(kBlockA), 0, s, P.ns, P.face.p,
                           w.h.p, P.z.p);
    }
    hipLaunchKernelGGL(k_normM, dim3(gf), dim3(kBlockA), 0, s, nf, m.fslot.p, m.farea.p, w.partial.p);
    HG_CHECK_HIP(hipGetLastError());
    double nm2, dummy;
    reduce_pair(m, w, gf, s, nm2, dummy);
    const double normM = sqrt(nm2);
    AdmmResult r;
    const bool fixed = iters > 0;
    const bool monitor = !fixed && depth >= 0;
    const int cap = fixed ? iters : o.max_admm;
    const int check = monitor ? std::max(64, o.check_every) : std::max(1, o.check_every);
    // iterations between two checks: one chunk, or kCoarseChecks chunks far
    // from convergence (DistStop)
    int interval = check, next_check = check;
    float *ga = w.g0.p, *gb = w.g1.p, *za = w.z0.p, *zb = w.z1.p;
    // algorithmic bytes of one iteration: per face g, h, its three twin
    // slots, copies and slot geometry (e, w) read, g and the copies written
    // (the neighbours' g and copies are the same arrays, read by their own
    // faces)
    r.bytes_per_iter = (uint64_t)168 * nf;
    // group kernels: the chunk sums read per slot its face, vector, area, g
    // and copy (48 B) and write 16 B per chunk; the fix reads per slot its
    // index, group, vector and copy and writes the copy (44 B), per face its
    // slot range, id, slots, z copies, h, old g and area and writes g (100 B)
    if (use_paths)
        r.bytes_per_iter += (uint64_t)92 * P.ns + (uint64_t)16 * P.nch + (uint64_t)100 * P.ng_face;
    RunTimer rt;
    int run_len = 0;
    DistStop stop;
    auto iterate = [&](float* gi, float* zi, float* go, float* zo) {
        if (!use_paths) {
            hipLaunchKernelGGL(k_admm_face, dim3(gf), dim3(kBlockA), 0, s, nf, m.twin.p, m.sgeo.p, w.h.p, gi, zi,
                               go, zo, mu, (float)o.relax);
        } else {
            hipLaunchKernelGGL(k_admm_face_paths, dim3(gf + P.nch), dim3(kBlockA), 0, s, nf, gf, P.nch, m.twin.p,
                               m.sgeo.p, m.farea.p, w.h.p, gi, zi, go, zo, P.chunk_path.p, P.cptr.p, P.ptr.p,
                               P.face.p, P.vec.p, P.z.p, P.pc.p, mu, (float)o.relax);
            hipLaunchKernelGGL(k_path_face_fix, dim3(grid_for(P.ng_face, kBlockA)), dim3(kBlockA), 0, s, P.ng_face,
                               P.fg_ptr.p, P.fg_id.p, P.fg_slot.p, P.spath.p, P.cptr.p, P.pc.p, P.vec.p, m.farea.p,
                               gi, P.z.p, m.fslot.p, zo, w.h.p, mu, (float)o.relax, go);
        }
    };
    // runs of `check` iterations between checks, one captured graph for every
    // full run (an even count leaves the double buffers in their roles)
    GraphChunk graph;
    const bool graphs = !fixed && o.use_graphs && (check % 2) == 0;
    int it = 0;
    while (it < cap) {
        const int n = std::min(check - it % check, cap - it);
        rt.start(s);
        if (graphs && n == check && !graph.tried)
            graph.capture(s, [&] {
                float *g1 = ga, *g2 = gb, *z1 = za, *z2 = zb;
                for (int k = 0; k < n; ++k) {
                    iterate(g1, z1, g2, z2);
                    std::swap(g1, g2);
                    std::swap(z1, z2);
                }
            });
        if (graphs && n == check && graph.ready()) {
            graph.launch(s);
        } else {
            for (int k = 0; k < n; ++k) {
                iterate(ga, za, gb, zb);
                std::swap(ga, gb);   // (ga, za) is now the current state, (gb, zb) the previous
                std::swap(za, zb);
            }
        }
        HG_CHECK_HIP(hipGetLastError());
        it += n;
        r.iters = it;
        run_len = n;
        r.kernel_ms += rt.stop(s);
        r.timed_launches += run_len;
        const bool want = it >= next_check || it == cap;
        if (!fixed && want) {
            bool done;
            if (monitor) {
                double delta, dmax;
                dist_change(m, w, HG_FORM_FACE, depth, nullptr, ga, stop.first, s, delta, dmax);
                done = stop.update(delta, dmax, o.tol_admm);
                // the seam only once the distance has settled
                if (done && o.tol_seam > 0.0) {
                    r.seam = seam_now(m, w, HG_FORM_FACE, nullptr, ga, s) / m.hbar;
                    done = r.seam <= o.tol_seam;
                }
                if (!done && interval == check && stop.far(dmax, o.tol_admm)) {
                    interval = kCoarseChecks * check;
                    stop.restart();
                } else if (!done && interval > check && stop.near(dmax, o.tol_admm)) {
                    interval = check;
                    stop.restart();
                }
            } else {
                face_residuals(m, w, gf, gb, ga, zb, za, mu, o.relax, normM, s, r);
                done = r.rp <= o.tol_admm && r.rd <= o.tol_admm;
            }
            next_check = it + interval;
            if (done) {
                r.converged = true;
                break;
            }
        }
    }
    if (rt.open) {
        r.kernel_ms += rt.stop(s);
        r.timed_launches += run_len;
    }
    if (fixed) r.converged = true;
    if (monitor && !stop.first && o.tol_seam <= 0.0) r.seam = seam_now(m, w, HG_FORM_FACE, nullptr, ga, s) / m.hbar;
    if (r.iters > 0) face_residuals(m, w, gf, gb, ga, zb, za, mu, o.relax, normM, s, r);
    HG_CHECK_HIP(hipMemcpyAsync(w.gf.p, ga, (size_t)3 * nf * sizeof(float), hipMemcpyDeviceToDevice, s));
    r.launches = r.iters;
    return r;
}

}  // namespace hg
