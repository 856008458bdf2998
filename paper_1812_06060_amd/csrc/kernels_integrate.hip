// Integration of the optimised gradients into distances (Sec. 3.3, Sec. 4).
//
// The paper fixes d = 0 at the sources and walks the breadth-first sets
// D_1, D_2, ... in order: a vertex v_j takes the value of its partner v_k in
// D_{i-1} plus the change along the edge (j, k) -- Eq. 17 for face gradients
// (the mean of g_l . (p_j - p_k) over the faces containing the edge), or the
// edge difference +-x_e for the edge form.  So d(v_j) is the sum of the
// changes along the partner chain from v_j to its source.
//
// Here that sum is formed by pointer jumping: every vertex holds (s, p) =
// (sum of changes to p, p), and one round replaces (s, p) by
// (s + s[p], p[p]); after ceil(log2(depth)) rounds p is the source and s the
// whole sum.  That needs ~log2(depth) launches instead of depth dependent
// steps.  Sums are carried as FP32 double-float pairs (hi, lo) with
// error-free two-sum, i.e. compensated summation; each edge change is formed
// in FP64 from FP32 gradients and FP64 positions and split into (hi, lo).
//
// The same integration also serves as the ADMM stopping monitor: the change
// of the whole distance field between two checks (see dist_change).
#include <cmath>

#include "hgeo_internal.h"

namespace hg {

constexpr int kBlockI = 256;

#pragma clang fp contract(off)
__device__ inline void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}
// (ah, al) + (bh, bl) in double-float arithmetic
__device__ inline void df_add(float ah, float al, float bh, float bl, float& rh, float& rl) {
    float s, e;
    two_sum(ah, bh, s, e);
    e += al + bl;
    float h = s + e;
    rl = e - (h - s);
    rh = h;
}

// The part of the mesh a distance check covers.  With bdue null, every
// vertex; else the vertices of the components with cdue[c] != 0, where
// bdue[b] says for the block of kBlockI vertices b whether none (0), all (1)
// or some (2, then decided per vertex) of its vertices are covered.  A
// vertex's partner chain stays in its component, so the integration of the
// covered components reads nothing the skipped vertices would write.
struct CheckDue {
    const uint8_t* bdue;
    const int32_t* comp;
    const uint8_t* cdue;
};
__device__ inline bool vertex_due(const CheckDue& d, int block, int j) {
    if (!d.bdue) return true;
    const uint8_t b = d.bdue[block];
    return b == 1 || (b == 2 && d.cdue[d.comp[j]] != 0);
}

// Per vertex block: 0 if none of its vertices' components is due, 1 if all
// are, 2 otherwise.
__global__ void k_block_due(int nv, const int32_t* comp, const uint8_t* cdue, uint8_t* bdue) {
    __shared__ int any_due, all_due;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (threadIdx.x == 0) {
        any_due = 0;
        all_due = 1;
    }
    __syncthreads();
    if (j < nv) {
        if (cdue[comp[j]] != 0)
            any_due = 1;
        else
            all_due = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) bdue[blockIdx.x] = any_due ? (all_due ? 1 : 2) : 0;
}

// Per vertex: the change along the edge to its partner, and the jump state.
__global__ void k_int_step(int nv, int form, const int32_t* level, const int32_t* parent, const int32_t* pedge,
                           const int32_t* ev, const int32_t* ef, const float* xe,
                           const int32_t* h01, EdgeX ex, const float* g, const double* px, const double* py,
                           const double* pz, float* shi, float* slo, int32_t* jp, CheckDue due) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nv || !vertex_due(due, blockIdx.x, j)) return;
    // the three per-vertex loads issued together (parent and edge are -1
    // on sources and unreached vertices, and not used there)
    const int lj = level[j];
    const int k = parent[j];
    const int e = pedge[j];
    if (lj <= 0) {
        shi[j] = lj == 0 ? 0.f : INFINITY;
        slo[j] = 0.f;
        jp[j] = lj == 0 ? j : -1;
        return;
    }
    double step;
    if (form == HG_FORM_EDGE) {
        double x;
        if (xe) {
            x = (double)xe[e];
        } else {   // formed here, as k_edge_x forms it
            // an edge has a side-1 slot exactly when it has a second face
            const int h0 = h01[2 * e], h1 = h01[2 * e + 1];
            x = (double)edge_x(ex.S[e], ex.z[h0], h1 >= 0 ? ex.z[h1] : 0.f, h1 < 0, ex.inv1mu);
        }
        step = (ev[2 * e + 1] == j) ? x : -x;
    } else {
        double d0 = px[j] - px[k], d1 = py[j] - py[k], d2 = pz[j] - pz[k];
        double acc = 0.0;
        int n = 0;
        for (int s = 0; s < 2; ++s) {
            int f = ef[2 * e + s];
            if (f < 0) continue;
            acc += (double)g[3 * f] * d0 + (double)g[3 * f + 1] * d1 + (double)g[3 * f + 2] * d2;
            ++n;
        }
        step = acc / (double)n;
    }
    float hi = (float)step;
    shi[j] = hi;
    slo[j] = (float)(step - (double)hi);
    jp[j] = k;
}

__global__ void k_int_jump(int nv, const float* shi, const float* slo, const int32_t* jp, float* shi2, float* slo2,
                           int32_t* jp2, CheckDue due) {
    const int b = xcd_block(blockIdx.x, gridDim.x);
    int j = b * blockDim.x + threadIdx.x;
    if (j >= nv || !vertex_due(due, b, j)) return;
    int p = jp[j];
    if (p < 0 || jp[p] == p) {
        // unreachable, a source, or already pointing at a source
        shi2[j] = shi[j];
        slo2[j] = slo[j];
        jp2[j] = p;
        return;
    }
    float h, l;
    df_add(shi[j], slo[j], shi[p], slo[p], h, l);
    shi2[j] = h;
    slo2[j] = l;
    jp2[j] = jp[p];
}

// d = s (the partner chain ends at a source, where d = 0); +inf if unreached
__global__ void k_int_out(int nv, const int32_t* perm_v, const int32_t* jp, const float* shi, const float* slo,
                          float* d_user) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nv) return;
    d_user[perm_v[j]] = jp[j] < 0 ? INFINITY : shi[j] + slo[j];
}

struct IntSums {
    float* hi;
    float* lo;
    int32_t* jp;
};

static IntSums integrate_sums(Mesh& m, Work& w, int form, int depth, const float* xe, const float* g, hipStream_t s,
                              const EdgeX* ex = nullptr, CheckDue due = CheckDue{nullptr, nullptr, nullptr}) {
    const int nv = (int)m.nv;
    w.shi0.alloc(nv);
    w.slo0.alloc(nv);
    w.shi1.alloc(nv);
    w.slo1.alloc(nv);
    w.jp0.alloc(nv);
    w.jp1.alloc(nv);
    const int grid = grid_for(nv, kBlockI);
    hipLaunchKernelGGL(k_int_step, dim3(grid), dim3(kBlockI), 0, s, nv, form, w.level.p, w.parent.p, w.pedge.p,
                       m.ev.p, m.ef.p, ex ? nullptr : xe, m.h01.p, ex ? *ex : EdgeX{nullptr, nullptr, 0.f},
                       g, m.px.p, m.py.p, m.pz.p, w.shi0.p, w.slo0.p, w.jp0.p, due);
    HG_CHECK_HIP(hipGetLastError());
    // after r rounds every vertex sums 2^r chain edges; sources stop the walk
    int rounds = 0;
    while ((1ll << rounds) < (long long)depth) ++rounds;
    float *ha = w.shi0.p, *la = w.slo0.p, *hb = w.shi1.p, *lb = w.slo1.p;
    int32_t *pa = w.jp0.p, *pb = w.jp1.p;
    for (int r = 0; r < rounds; ++r) {
        hipLaunchKernelGGL(k_int_jump, dim3(grid), dim3(kBlockI), 0, s, nv, ha, la, pa, hb, lb, pb, due);
        HG_CHECK_HIP(hipGetLastError());
        std::swap(ha, hb);
        std::swap(la, lb);
        std::swap(pa, pb);
    }
    return IntSums{ha, la, pa};
}

void integrate(Mesh& m, Work& w, int form, int depth, float* d_user, hipStream_t s) {
    IntSums r = integrate_sums(m, w, form, depth, w.xe.p, w.gf.p, s);
    hipLaunchKernelGGL(k_int_out, dim3(grid_for(m.nv, kBlockI)), dim3(kBlockI), 0, s, (int)m.nv, m.perm_v.p, r.jp,
                       r.hi, r.lo, d_user);
    HG_CHECK_HIP(hipGetLastError());
}

// ------------------------------------------------------- distance monitor
__device__ inline double blk_max2(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = sh[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = fmax(r, sh[i]);
    return r;
}

// partial[2b] = max |d - dprev|, partial[2b+1] = max |d| over reached
// vertices of block b; dprev <- d.
__global__ void k_dist_delta(int nv, const int32_t* jp, const float* shi, const float* slo, float* dprev,
                             int first, double* partial) {
    __shared__ double sh[kBlockI / 64];
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    double dl = 0.0, mx = 0.0;
    if (j < nv && jp[j] >= 0) {
        float d = shi[j] + slo[j];
        dl = first ? INFINITY : fabs((double)d - (double)dprev[j]);
        mx = fabs((double)d);
        dprev[j] = d;
    }
    dl = blk_max2(dl, sh);
    mx = blk_max2(mx, sh);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = dl;
        partial[2 * blockIdx.x + 1] = mx;
    }
}

// Per connected component: the largest |d - d_prev| and the largest d, as
// atomic maxima on the bit patterns (non-negative doubles order as their
// bits).  A block whose vertices lie in one component (the usual case: the
// components of a joined batch are contiguous) reduces first.
__global__ void k_dist_delta_comp(int nv, const int32_t* jp, const float* shi, const float* slo, float* dprev,
                                  int first, const int32_t* comp, unsigned long long* comp_pair, CheckDue due) {
    __shared__ double sh[kBlockI / 64];
    __shared__ int c_first, mixed;
    if (due.bdue && due.bdue[blockIdx.x] == 0) return;   // the whole block
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    double dl = 0.0, mx = 0.0;
    int c = -1;
    if (j < nv && vertex_due(due, blockIdx.x, j)) {
        c = comp[j];
        if (jp[j] >= 0) {
            float d = shi[j] + slo[j];
            dl = first ? INFINITY : fabs((double)d - (double)dprev[j]);
            mx = fabs((double)d);
            dprev[j] = d;
        }
    }
    if (threadIdx.x == 0) {
        c_first = c;
        mixed = 0;
    }
    __syncthreads();
    if (c >= 0 && c != c_first) mixed = 1;
    __syncthreads();
    if (!mixed) {
        dl = blk_max2(dl, sh);
        mx = blk_max2(mx, sh);
        if (threadIdx.x == 0 && c_first >= 0) {
            atomicMax(&comp_pair[2 * c_first], (unsigned long long)__double_as_longlong(dl));
            atomicMax(&comp_pair[2 * c_first + 1], (unsigned long long)__double_as_longlong(mx));
        }
    } else if (c >= 0) {
        atomicMax(&comp_pair[2 * c], (unsigned long long)__double_as_longlong(dl));
        atomicMax(&comp_pair[2 * c + 1], (unsigned long long)__double_as_longlong(mx));
    }
}

__global__ void k_zero_u64(int n, unsigned long long* a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0ull;
}

__global__ void k_reduce_pairs_max(double* partial, int n) {
    __shared__ double sh[kBlockI / 64];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        a = fmax(a, partial[2 * i]);
        b = fmax(b, partial[2 * i + 1]);
    }
    a = blk_max2(a, sh);
    b = blk_max2(b, sh);
    if (threadIdx.x == 0) {
        partial[2 * n] = a;
        partial[2 * n + 1] = b;
    }
}

// Largest disagreement over the edges between the integrated distance and
// the optimised field, |d_head - d_tail - x_e| (face form: x_e = the mean of
// g_f . (p_head - p_tail) over the edge's faces).  It is zero on the edges
// the integration followed; elsewhere it is the jump of d across the edge
// left by what is still not a gradient in the field, the seam between
// branches of the breadth-first tree.  partial[block] = the block's largest.
__global__ void k_seam(int ne, const int32_t* ev, const int32_t* ef, const int32_t* level, const float* d,
                       const float* xe, const float* g, const double* px, const double* py, const double* pz,
                       double* partial) {
    __shared__ double sh[kBlockI / 64];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    double sm = 0.0;
    if (e < ne) {
        const int a = ev[2 * e], b = ev[2 * e + 1];
        if (level[a] >= 0 && level[b] >= 0) {
            double x = 0.0;
            if (xe) {
                x = xe[e];
            } else {
                const double dx = px[b] - px[a], dy = py[b] - py[a], dz = pz[b] - pz[a];
                int n = 0;
                for (int q = 0; q < 2; ++q) {
                    const int f = ef[2 * e + q];
                    if (f < 0) continue;
                    x += (double)g[3 * f] * dx + (double)g[3 * f + 1] * dy + (double)g[3 * f + 2] * dz;
                    ++n;
                }
                x /= n;
            }
            sm = fabs((double)d[b] - (double)d[a] - x);
        }
    }
    sm = blk_max2(sm, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = sm;
}

void dist_change(Mesh& m, Work& w, int form, int depth, const float* xe, const float* g, bool first, hipStream_t s,
                 double& delta, double& dmax, double* seam, const EdgeX* ex) {
    const int nv = (int)m.nv;
    w.dprev.alloc(nv);
    const int grid = grid_for(nv, kBlockI);
    if ((int)w.partial.n < 2 * grid + 8) w.partial.alloc((size_t)2 * grid + 8);
    IntSums r = integrate_sums(m, w, form, depth, xe, g, s, ex);
    hipLaunchKernelGGL(k_dist_delta, dim3(grid), dim3(kBlockI), 0, s, nv, r.jp, r.hi, r.lo, w.dprev.p,
                       first ? 1 : 0, w.partial.p);
    hipLaunchKernelGGL(k_reduce_pairs_max, dim3(1), dim3(kBlockI), 0, s, w.partial.p, grid);
    HG_CHECK_HIP(hipGetLastError());
    HG_CHECK_HIP(hipMemcpyAsync(w.pinned, w.partial.p + 2 * grid, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HG_CHECK_HIP(hipStreamSynchronize(s));
    delta = w.pinned[0];
    dmax = w.pinned[1];
    if (seam) *seam = seam_now(m, w, form, xe, g, s);
}

void dist_change_comp(Mesh& m, Work& w, int form, int depth, const float* xe, const float* g, bool first,
                      hipStream_t s, std::vector<double>& delta, std::vector<double>& dmax, const EdgeX* ex,
                      const uint8_t* due) {
    const int nv = (int)m.nv, nc = std::max(1, m.n_comp);
    const int grid = grid_for(nv, kBlockI);
    w.dprev.alloc(nv);
    w.comp_pair.alloc((size_t)2 * nc);
    CheckDue cd{nullptr, nullptr, nullptr};
    if (due) {
        w.cdue.alloc((size_t)nc);
        w.bdue.alloc((size_t)grid);
        // the stream is synchronised below, before the host array can change
        HG_CHECK_HIP(hipMemcpyAsync(w.cdue.p, due, (size_t)nc, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_block_due, dim3(grid), dim3(kBlockI), 0, s, nv, m.comp_v.p, w.cdue.p, w.bdue.p);
        HG_CHECK_HIP(hipGetLastError());
        cd = CheckDue{w.bdue.p, m.comp_v.p, w.cdue.p};
    }
    IntSums r = integrate_sums(m, w, form, depth, xe, g, s, ex, cd);
    hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(2 * nc, kBlockI)), dim3(kBlockI), 0, s, 2 * nc,
                       reinterpret_cast<unsigned long long*>(w.comp_pair.p));
    hipLaunchKernelGGL(k_dist_delta_comp, dim3(grid), dim3(kBlockI), 0, s, nv, r.jp, r.hi, r.lo, w.dprev.p,
                       first ? 1 : 0, m.comp_v.p, reinterpret_cast<unsigned long long*>(w.comp_pair.p), cd);
    HG_CHECK_HIP(hipGetLastError());
    std::vector<double> h((size_t)2 * nc);
    HG_CHECK_HIP(hipMemcpyAsync(h.data(), w.comp_pair.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HG_CHECK_HIP(hipStreamSynchronize(s));
    delta.resize(nc);
    dmax.resize(nc);
    for (int c = 0; c < nc; ++c) {
        delta[c] = h[2 * c];
        dmax[c] = h[2 * c + 1];
    }
}

double seam_now(Mesh& m, Work& w, int form, const float* xe, const float* g, hipStream_t s) {
    const int ge = grid_for(m.ne, kBlockI);
    if ((int)w.partial.n < ge + 8) w.partial.alloc((size_t)ge + 8);
    hipLaunchKernelGGL(k_seam, dim3(ge), dim3(kBlockI), 0, s, (int)m.ne, m.ev.p, m.ef.p, w.level.p, w.dprev.p,
                       form == HG_FORM_EDGE ? xe : nullptr, g, m.px.p, m.py.p, m.pz.p, w.partial.p);
    HG_CHECK_HIP(hipGetLastError());
    return reduce_partials(m, w, ge, true, s);
}

}  // namespace hg
