// LDS-tiled diffusion sweeps for (A - t L_c) u = u_0 (Eq. 4, update Eq. 7).
//
// A tile is a connected patch of at most 1024 vertices (a contiguous range
// of internal vertex ids) plus its halo (the outside one-ring).  A workgroup
// loads its tile and halo into LDS once, performs `inner` Jacobi sweeps of
// the tile with the halo held fixed, and writes the tile back, so
// information crosses a whole tile per HBM round trip instead of one ring,
// which is what a relative-accuracy solve of a field that decays by ~e^-1
// per ring needs (plain sweeps would need more than the breadth-first depth).
//
// One global pass runs the tiles colour by colour (the tiles are coloured
// at mesh creation so that no tile's halo lies in a tile of its own colour):
// each colour's launch updates its tiles in place from the latest values of
// the other colours -- block Gauss-Seidel between tiles, about 40% fewer
// passes than updating all tiles from the previous pass.  Tiles of one
// colour never read each other, so a launch's result does not depend on
// workgroup timing.  The fixed point is unchanged: when every tile is
// converged for its converged halo, Eq. 7 holds everywhere.
//
// Range: during a pass every vertex j carries a reference exponent R_j and
// LDS holds u_j 2^-R_j.  R_j starts at the exponent of u_j (none if u_j = 0)
// and is raised by a max-plus relaxation, R_j >= R_k + floor(log2 c_jk) - 2
// over the tile's edges, so that every rescaled weight c_jk 2^(R_k - R_j)
// is at most 8: a vertex whose stored value is stale by many binades, or one
// the front reaches during this pass, can then grow only by a bounded factor
// per sweep, for any t.  The rescaling is by exact powers of two, so
// rounding is that of FP64 on u_j 2^-R_j.

// Coefficients c_jk = t theta_jk / (A_j + t sum_k theta_jk) and the LDS
// slots of the neighbours stay in registers for the whole pass; the
// tile-local neighbour table is in ELL layout (slot-major, coalesced).
#include <climits>
#include <cmath>

#include "hgeo_internal.h"

namespace hg {

constexpr int kTile = 1024;    // vertices per tile at most (mesh_create uses the same)
constexpr int kThreads = 1024;  // one vertex per thread: few registers (52), high occupancy
constexpr int kPer = kTile / kThreads;

__device__ inline double blk_max(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = sh[0];
    for (int i = 1; i < kThreads / 64; ++i) r = fmax(r, sh[i]);
    return r;
}
constexpr int kNone = -(1 << 30);   // "no reference exponent yet"

// OV: overlapping tiles.  Then halo slots [0, n_ov) hold overlap vertices,
// updated by the sweeps like the core (overlap vertex tid is a second row of
// thread tid, with its coefficients and neighbour slots kept in LDS rather
// than registers, so that two workgroups still fit per compute unit), and
// only the slots from n_ov on are held fixed; the core alone is written
// back.  Without OV every halo slot is fixed.
__host__ __device__ constexpr size_t ov_lds_offset(int ntot) { return ((size_t)ntot * 20 + 7) & ~(size_t)7; }

// theta is staged through LDS in chunks of this many rows of kTile doubles
// (48 KB at valence 6, 64 KB at 8 and above)
__host__ __device__ constexpr int theta_stage_width(int maxw) { return maxw < 8 ? maxw : 8; }

template <int MAXW, bool OV>
__device__ __forceinline__ void patch_pass_body(
    const int32_t* __restrict__ tile_list, const double* __restrict__ tile_t, const int32_t* __restrict__ tile_ptr,
    const int32_t* __restrict__ halo_ptr, const int32_t* __restrict__ halo_idx, const int32_t* __restrict__ n_ov,
    const int32_t* __restrict__ ell_ptr, const uint8_t* __restrict__ ell_width, const uint16_t* __restrict__ lnb,
    const int32_t* __restrict__ tile_k0, const int32_t* __restrict__ row_ptr, const double* __restrict__ theta,
    const double* __restrict__ invD, const int32_t* __restrict__ level, const double* vin, const int32_t* ein,
    double* vout, int32_t* eout, int inner, double* __restrict__ partial) {
    extern __shared__ double lds[];
    __shared__ double shd[kThreads / 64];
    const int p = tile_list[xcd_block(blockIdx.x, gridDim.x)];
    const double t = tile_t[p];   // the diffusion time of the tile's component
    const int v0 = tile_ptr[p];
    const int np = tile_ptr[p + 1] - v0;
    const int h0 = halo_ptr[p], nh = halo_ptr[p + 1] - h0;
    const int no = OV ? n_ov[p] : 0;
    const int ntot = kTile + nh;
    double* cur = lds;
    double* nxt = lds + ntot;
    int* R = reinterpret_cast<int*>(lds + 2 * ntot);
    // overlap rows' coefficients and neighbour slots, slot-major (s * no + j)
    double* oc = OV ? reinterpret_cast<double*>(reinterpret_cast<char*>(lds) + ov_lds_offset(ntot)) : nullptr;
    uint16_t* ol = OV ? reinterpret_cast<uint16_t*>(oc + MAXW * no) : nullptr;
    const int tid = threadIdx.x;

    // 1. coefficients c_jk = t theta_jk / (A_j + t sum theta) into registers,
    //    with floor(log2 |c_jk|) for the exponent relaxation below
    const int W = ell_width[p];
    const int eb = ell_ptr[p];
    double c[kPer][MAXW];
    uint16_t l[kPer][MAXW];
    double b[kPer];
    int Rown[kPer];
    // The ELL row lists the CSR row in order, and the tile's CSR rows are
    // one contiguous range of theta: it is read coalesced into LDS (which
    // holds no state yet), at once for valence <= 8, and each thread picks
    // its row from there.
    const int K0 = tile_k0[p];
    const int nk = tile_k0[p + 1] - K0;
    // Everything a pass reads from HBM is requested here, before the first
    // barrier, so the loads overlap: the tables, theta, the core's state and
    // this thread's first fixed-ring entry (the rest, rare, is read where it
    // is used).  Tiles of one colour never write what another reads, so the
    // state read now is the state at any point of the pass.
    const int ih = tid + no;   // this thread's first fixed-ring entry
    const bool hh = ih < nh;
    const int hgl = hh ? halo_idx[h0 + ih] : 0;
    int k0[kPer];
    uint32_t okm[kPer];   // bit s: slot s is a neighbour
    double vown[kPer];
    int eown[kPer], lown[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        int i = tid + q * kThreads;
        const bool in = i < np;
        b[q] = in ? invD[v0 + i] : 0.0;
        k0[q] = in ? row_ptr[v0 + i] - K0 : 0;
        vown[q] = in ? vin[v0 + i] : 0.0;
        eown[q] = in ? ein[v0 + i] : 0;
        lown[q] = in ? level[v0 + i] : -1;
        okm[q] = 0;
#pragma unroll
        for (int s = 0; s < MAXW; ++s) {
            bool ok = in && (s < W);
            uint16_t li = ok ? lnb[eb + s * kTile + i] : (uint16_t)0xFFFF;
            ok = ok && li != 0xFFFF;
            l[q][s] = ok ? li : (uint16_t)0;   // padding reads slot 0 with weight 0
            okm[q] |= ok ? (1u << s) : 0u;
            c[q][s] = 0.0;
        }
    }
    const double hv = hh ? vin[hgl] : 0.0;
    const int he = hh ? ein[hgl] : 0;
    constexpr int kChunk = theta_stage_width(MAXW) * kTile;   // doubles
    for (int cb = 0; cb < nk; cb += kChunk) {
        const int nc = min(kChunk, nk - cb);
        if (cb > 0) __syncthreads();
        double th[kChunk / kThreads];
#pragma unroll
        for (int j = 0; j < kChunk / kThreads; ++j) {
            const int k = tid + j * kThreads;
            th[j] = k < nc ? theta[K0 + cb + k] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < kChunk / kThreads; ++j) {
            const int k = tid + j * kThreads;
            if (k < nc) lds[k] = th[j];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
#pragma unroll
            for (int s = 0; s < MAXW; ++s) {
                const int kk = k0[q] + s - cb;
                if (((okm[q] >> s) & 1u) && kk >= 0 && kk < nc) c[q][s] = t * lds[kk] * b[q];
            }
        }
    }
    __syncthreads();   // the chunks' LDS is reused below
    // the overlap row of this thread (OV): vertex halo_idx[h0 + tid], tid < no
    const bool has1 = OV && tid < no;
    const int g1 = has1 ? halo_idx[h0 + tid] : 0;
    double b1 = 0.0;
    int Rown1 = kNone;
    if (has1) {
        const double id = invD[g1];
        const int k0 = row_ptr[g1];
        b1 = id;
        const int ob = eb + W * kTile;
        for (int s = 0; s < MAXW; ++s) {
            bool ok = s < W;
            uint16_t li = ok ? lnb[ob + s * no + tid] : (uint16_t)0xFFFF;
            ok = ok && li != 0xFFFF;
            ol[s * no + tid] = ok ? li : (uint16_t)0;
            oc[s * no + tid] = ok ? t * theta[k0 + s] * id : 0.0;
        }
    }

    // 2. reference exponents: own exponent for non-zero values (and the
    //    source term's for sources), "none" otherwise; the fixed halo keeps
    //    its own
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        int i = tid + q * kThreads;
        int r = kNone;
        if (i < np) {
            if (vown[q] != 0.0) r = eown[q];
            if (lown[q] == 0) r = max(r, ilogb(b[q]));
        }
        Rown[q] = r;
        R[i] = r;
    }
    if (has1) {
        int r = kNone;
        if (vin[g1] != 0.0) r = ein[g1];
        if (level[g1] == 0) r = max(r, ilogb(b1));
        Rown1 = r;
        R[kTile + tid] = r;
    }
    if (hh) R[kTile + ih] = hv != 0.0 ? he : kNone;
    for (int i = ih + kThreads; i < nh; i += kThreads) {
        int g = halo_idx[h0 + i];
        R[kTile + i] = vin[g] != 0.0 ? ein[g] : kNone;
    }
    __syncthreads();
    // 3. max-plus relaxation R_j = max(R_j, R_k + floor(log2 |c_jk|) - 2) over
    //    the updated slots (fixed halo held).  Every weight c_jk 2^(R_k - R_j)
    //    is then <= 8, so no value can overflow within the pass.  The least
    //    fixed point is unique (all edge weights are negative), so the
    //    in-place, any-order updates give the same R every time; it is
    //    reached within as many rounds as there are updated slots.
    const int nrounds = kTile + no;
    for (int round = 0; round < nrounds; ++round) {
        int changed = 0;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            int i = tid + q * kThreads;
            if (i >= np) continue;
            int r = Rown[q];
#pragma unroll
            for (int s = 0; s < MAXW; ++s) {
                if (c[q][s] == 0.0) continue;
                int rk = R[l[q][s]];
                if (rk == kNone) continue;
                r = max(r, rk + ilogb(c[q][s]) - 2);
            }
            if (r != Rown[q]) {
                Rown[q] = r;
                R[i] = r;
                changed = 1;
            }
        }
        if (has1) {
            int r = Rown1;
            for (int s = 0; s < W; ++s) {
                const double cs = oc[s * no + tid];
                if (cs == 0.0) continue;
                int rk = R[ol[s * no + tid]];
                if (rk == kNone) continue;
                r = max(r, rk + ilogb(cs) - 2);
            }
            if (r != Rown1) {
                Rown1 = r;
                R[kTile + tid] = r;
                changed = 1;
            }
        }
        if (!__syncthreads_or(changed)) break;
    }
    // 4. values and weights relative to the reference exponents
    double vstart[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        int i = tid + q * kThreads;
        const int rj = Rown[q];
        const bool live = i < np && rj != kNone;
        double x = 0.0;
        if (live) {
            if (vown[q] != 0.0) x = ldexp(vown[q], eown[q] - rj);
            b[q] = lown[q] == 0 ? ldexp(b[q], -rj) : 0.0;
        } else {
            b[q] = 0.0;
        }
#pragma unroll
        for (int s = 0; s < MAXW; ++s) {
            int rk = R[l[q][s]];
            c[q][s] = (live && c[q][s] != 0.0 && rk != kNone) ? ldexp(c[q][s], rk - rj) : 0.0;
        }
        vstart[q] = x;
        cur[i] = x;   // slots np..kTile-1 of a short tile stay 0
    }
    if (has1) {
        const int rj = Rown1;
        const bool live = rj != kNone;
        double x = 0.0;
        if (live) {
            double v = vin[g1];
            if (v != 0.0) x = ldexp(v, ein[g1] - rj);
            b1 = level[g1] == 0 ? ldexp(b1, -rj) : 0.0;
        } else {
            b1 = 0.0;
        }
        for (int s = 0; s < W; ++s) {
            const double cs = oc[s * no + tid];
            const int rk = R[ol[s * no + tid]];
            oc[s * no + tid] = (live && cs != 0.0 && rk != kNone) ? ldexp(cs, rk - rj) : 0.0;
        }
        cur[kTile + tid] = x;
    }
    if (hh) {
        cur[kTile + ih] = hv;   // the fixed halo's reference exponent is its own
        nxt[kTile + ih] = hv;
    }
    for (int i = ih + kThreads; i < nh; i += kThreads) {
        double v = vin[halo_idx[h0 + i]];
        cur[kTile + i] = v;
        nxt[kTile + i] = v;
    }
    __syncthreads();

    // 5. inner Jacobi sweeps in LDS
    for (int it = 0; it < inner; ++it) {
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            int i = tid + q * kThreads;
            double acc = b[q];
#pragma unroll
            for (int s = 0; s < MAXW; ++s) acc = fma(c[q][s], cur[l[q][s]], acc);
            if (i < np) nxt[i] = acc;
        }
        if (has1) {
            double acc = b1;
            for (int s = 0; s < W; ++s) acc = fma(oc[s * no + tid], cur[ol[s * no + tid]], acc);
            nxt[kTile + tid] = acc;
        }
        __syncthreads();
        double* tmp = cur;
        cur = nxt;
        nxt = tmp;
    }

    // 6. write back the core renormalised; largest relative change over the
    //    pass (a non-finite value would be a bug: report it as not converged)
    double res = 0.0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        int i = tid + q * kThreads;
        if (i >= np) continue;
        const int g = v0 + i;
        double x = cur[i];
        if (!isfinite(x)) {
            vout[g] = 0.0;
            eout[g] = 0;
            res = 1e300;
        } else if (x == 0.0) {
            vout[g] = 0.0;
            eout[g] = 0;
            if (lown[q] >= 0) res = 1.0;
        } else {
            int ex = ilogb(x);
            vout[g] = ldexp(x, -ex);
            eout[g] = Rown[q] + ex;
            res = fmax(res, vstart[q] == 0.0 ? 1.0 : fabs(x - vstart[q]) / fabs(x));
        }
    }
    res = blk_max(res, shd);
    if (tid == 0) partial[p] = res;
}

#define HG_PATCH_PARAMS                                                                                           \
    const int32_t *__restrict__ tile_list, const double *__restrict__ tile_t, const int32_t *__restrict__ tile_ptr, \
        const int32_t *__restrict__ halo_ptr, const int32_t *__restrict__ halo_idx,                                 \
        const int32_t *__restrict__ n_ov, const int32_t *__restrict__ ell_ptr,                                      \
        const uint8_t *__restrict__ ell_width, const uint16_t *__restrict__ lnb,                                    \
        const int32_t *__restrict__ tile_k0, const int32_t *__restrict__ row_ptr, const double *__restrict__ theta,  \
        const double *__restrict__ invD, const int32_t *__restrict__ level, const double *vin, const int32_t *ein,   \
        double *vout, int32_t *eout, int inner, double *__restrict__ partial
#define HG_PATCH_FWD                                                                                       \
    tile_list, tile_t, tile_ptr, halo_ptr, halo_idx, n_ov, ell_ptr, ell_width, lnb, tile_k0, row_ptr, theta, invD, \
        level, vin, ein, vout, eout, inner, partial

// plain tiles: held to 64 registers up to valence 8 so that two workgroups
// fit per CU (55 at valence 6); registers as needed beyond
template <int MAXW>
__global__ void __launch_bounds__(kThreads, MAXW <= 8 ? 8 : 4) k_patch_pass(HG_PATCH_PARAMS) {
    patch_pass_body<MAXW, false>(HG_PATCH_FWD);
}
// overlapping tiles: held to 64 registers so that two workgroups fit per CU
template <int MAXW>
__global__ void __launch_bounds__(kThreads, 8) k_patch_pass_ov(HG_PATCH_PARAMS) {
    patch_pass_body<MAXW, true>(HG_PATCH_FWD);
}
#undef HG_PATCH_PARAMS
#undef HG_PATCH_FWD

static size_t patch_lds_bytes(int max_halo) { return (size_t)(kTile + max_halo) * (8 + 8 + 4); }
// overlapping tiles: the above (aligned), plus per overlap row maxw
// coefficients (FP64) and neighbour slots (uint16)
static size_t patch_lds_bytes_ov(int max_halo, int max_ov, int maxw) {
    return ov_lds_offset(kTile + max_halo) + (size_t)max_ov * maxw * (8 + 2);
}
static int template_width(int w) { return w <= 6 ? 6 : (w <= 8 ? 8 : 16); }

// valence within the register tables, LDS within 64 KiB
bool patch_supported(const Mesh& m) {
    return m.max_ell_width <= 16 && m.patch_size == kTile && patch_lds_bytes(m.max_halo) <= 65536;
}

// Runs patch passes until the largest relative change over a pass is <= tol;
// overlap > 0: on the overlapping tiles with that many rings (one overlap
// vertex per thread at most).
DiffusionResult run_diffusion_patch(Mesh& m, Work& w, const hg_opts& o, int inner, hipStream_t s, int overlap) {
    const int nv = (int)m.nv;
    const int nt = m.n_patches;
    if ((int)w.partial.n < nt + 8) w.partial.alloc((size_t)nt + 8);
    const Mesh::OverlapTileSet* ot = nullptr;
    if (overlap > 0) {
        ot = m.ensure_overlap_tiles(overlap, kThreads, 65536, template_width(m.max_ell_width), s);
        if (!ot) throw Error{HG_E_INVALID_ARG, "overlapping tiles do not fit this mesh (more overlap vertices than "
                                               "threads); use fewer overlap rings"};
        if (ot->max_ell_width > 16 ||
            patch_lds_bytes_ov(ot->max_halo, ot->max_ov, template_width(ot->max_ell_width)) > 65536)
            throw Error{HG_E_INVALID_ARG, "overlapping tiles exceed the valence or LDS limits"};
    }
    const int maxw = ot ? ot->max_ell_width : m.max_ell_width;
    // the region, or theta's staging before it, whichever is larger (<= 64 KiB)
    const size_t lds = std::max(ot ? patch_lds_bytes_ov(ot->max_halo, ot->max_ov, template_width(maxw))
                                   : patch_lds_bytes(m.max_halo),
                                (size_t)theta_stage_width(template_width(maxw)) * kTile * sizeof(double));
    const std::vector<int32_t>& color_ptr = ot ? ot->color_ptr_host : m.color_ptr_host;
    const int32_t* order = ot ? ot->tile_order.p : m.tile_order.p;
    const int32_t* halo_ptr = ot ? ot->halo_ptr.p : m.halo_ptr.p;
    const int32_t* halo_idx = ot ? ot->halo_idx.p : m.halo_idx.p;
    const int32_t* n_ov = ot ? ot->n_ov.p : nullptr;
    const int32_t* ell_ptr = ot ? ot->ell_ptr.p : m.ell_ptr.p;
    const uint8_t* ell_width = ot ? ot->ell_width.p : m.ell_width.p;
    const uint16_t* lnb = ot ? ot->lnb.p : m.lnb.p;
    DiffusionResult r;
    // algorithmic bytes of one pass: tile tables (ELL slots), theta and
    // row offsets of the CSR rows, halo list, 1/D and level, (v, e) read for
    // tile and halo, (v, e) written; overlap vertices also read their 1/D,
    // level, row offset and theta
    const uint64_t ell_n = ot ? ot->lnb.n : m.lnb.n;
    const uint64_t halo_n = ot ? ot->halo_idx.n : m.halo_idx.n;
    r.bytes_per_pass = ell_n * 2 + (uint64_t)m.col.n * 8 + halo_n * (4 + 16) + (uint64_t)nv * (4 + 8 + 4 + 12 + 12) +
                       (uint64_t)nt * (ot ? 21 : 17);
    // overlap rows: their 1/D, level and row offset, and theta for the ELL
    // entries beyond the plain tiles' (the overlap rows' slots)
    if (ot) r.bytes_per_pass += halo_n * 12 + (ell_n > m.lnb.n ? (ell_n - m.lnb.n) * 8 : 0);
    double* va = w.v0.p;   // updated in place
    int32_t* ea = w.e0.p;
    const int check = std::max(1, o.check_every / std::max(1, inner / 4));
    const int max_passes = std::max(1, o.max_sweeps / std::max(1, inner));
    // one pass = the colours in order, each updating its tiles in place from
    // the latest values of the others (block Gauss-Seidel between tiles,
    // Jacobi within a colour: tiles of one colour are independent)
    auto pass = [&] {
        for (size_t c = 0; c + 1 < color_ptr.size(); ++c) {
            const int c0 = color_ptr[c], nc = color_ptr[c + 1] - c0;
            if (nc == 0) continue;
#define HG_PATCH_ARGS                                                                                           \
    dim3(nc), dim3(kThreads), lds, s, order + c0, w.tile_t.p, m.tile_ptr.p, halo_ptr, halo_idx, n_ov, ell_ptr, \
        ell_width, lnb, m.tile_k0.p, m.row_ptr.p, m.theta.p, w.invD.p, w.level.p, va, ea, va, ea, inner, w.partial.p
            if (ot) {
                if (maxw <= 6)
                    hipLaunchKernelGGL(k_patch_pass_ov<6>, HG_PATCH_ARGS);
                else if (maxw <= 8)
                    hipLaunchKernelGGL(k_patch_pass_ov<8>, HG_PATCH_ARGS);
                else
                    hipLaunchKernelGGL(k_patch_pass_ov<16>, HG_PATCH_ARGS);
            } else {
                if (maxw <= 6)
                    hipLaunchKernelGGL(k_patch_pass<6>, HG_PATCH_ARGS);
                else if (maxw <= 8)
                    hipLaunchKernelGGL(k_patch_pass<8>, HG_PATCH_ARGS);
                else
                    hipLaunchKernelGGL(k_patch_pass<16>, HG_PATCH_ARGS);
            }
#undef HG_PATCH_ARGS
        }
    };
    // runs of `check` passes between checks, captured once into a graph
    GraphChunk graph;
    RunTimer rt;
    int it = 0;
    while (it < max_passes) {
        const int n = std::min(check, max_passes - it);
        rt.start(s);
        if (o.use_graphs && n == check && !graph.tried)
            graph.capture(s, [&] {
                for (int k = 0; k < n; ++k) pass();
            });
        if (o.use_graphs && n == check && graph.ready()) {
            graph.launch(s);
        } else {
            for (int k = 0; k < n; ++k) pass();
        }
        HG_CHECK_HIP(hipGetLastError());
        it += n;
        r.passes = it;
        r.sweeps = it * inner;
        r.kernel_ms += rt.stop(s);
        r.timed_launches += n;
        r.res = reduce_partials(m, w, nt, true, s);
        if (r.res <= o.tol_u) {
            r.converged = true;
            break;
        }
    }
    return r;
}

}  // namespace hg
