// Queries on several resident meshes in one solve (Algorithm 1 run once for
// all of them; Sec. 5.2's source sets per mesh).
//
// The meshes are joined on the device into one mesh whose connected
// components they are: every array is the concatenation of the members'
// arrays, with vertex, face, edge, slot, tile, halo, neighbour-table and
// component indices shifted by the sizes of the members before it.  Nothing
// is rebuilt on the host: the members' tiles, colours, one-ring tables and
// cotangent weights are reused as they are, and the tiles of colour c of
// every member form colour c of the join (members share no vertex, so the
// tiles of one colour stay independent).  Internal and caller orders are
// both concatenations, so member i's caller vertex v is the join's caller
// vertex v + (vertices of the members before i), and likewise for faces and
// canonical edges.  A solve on the join with a diffusion time per component
// gives every member the result it has alone (to the tolerances of the
// solve, whose stopping rules see the whole join).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>

#include "hgeo_internal.h"

namespace hg {

constexpr int kBlockU = 256;

// out[i] = in[i] + add, except that negative entries stay as they are when
// keep_neg is set (the "none" markers of twin slots and edge faces)
__global__ void k_shift_i32(int64_t n, const int32_t* __restrict__ in, int32_t* __restrict__ out, int32_t add,
                            int keep_neg) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t x = in[i];
    out[i] = (keep_neg && x < 0) ? x : x + add;
}

template <class T>
static void copy_into(DBuf<T>& dst, size_t at, const DBuf<T>& src, size_t count, hipStream_t s) {
    if (count == 0) return;
    if (!src.p || src.n < count) throw Error{HG_E_DEVICE, "join: member array smaller than expected"};
    HG_CHECK_HIP(hipMemcpyAsync(dst.p + at, src.p, count * sizeof(T), hipMemcpyDeviceToDevice, s));
}

static void shift_into(int32_t* dst, size_t at, const int32_t* src, size_t count, int64_t add, bool keep_neg,
                       hipStream_t s) {
    if (count == 0) return;
    if (add > INT32_MAX) throw Error{HG_E_INVALID_ARG, "join: index beyond int32"};
    hipLaunchKernelGGL(k_shift_i32, dim3(grid_for((int64_t)count, kBlockU)), dim3(kBlockU), 0, s, (int64_t)count, src,
                       dst + at, (int32_t)add, keep_neg ? 1 : 0);
    HG_CHECK_HIP(hipGetLastError());
}

std::unique_ptr<Mesh> join_meshes(const std::vector<Mesh*>& parts, hipStream_t s) {
    if (parts.empty()) throw Error{HG_E_INVALID_ARG, "join: no meshes"};
    const Mesh& p0 = *parts[0];
    for (const Mesh* p : parts) {
        if (p->device != p0.device) throw Error{HG_E_INVALID_ARG, "batch meshes live on different devices"};
        if (p->patch_size != p0.patch_size) throw Error{HG_E_INVALID_ARG, "batch meshes have different tile sizes"};
        if (p->intrinsic != p0.intrinsic)
            throw Error{HG_E_INVALID_ARG, "a batch cannot mix intrinsic and extrinsic meshes"};
    }
    const size_t n = parts.size();
    // offsets of each member
    std::vector<int64_t> vo(n + 1, 0), fo(n + 1, 0), eo(n + 1, 0), to(n + 1, 0), ho(n + 1, 0), lo(n + 1, 0),
        co(n + 1, 0), ko(n + 1, 0), ceo(n + 1, 0), cfo(n + 1, 0), ao(n + 1, 0);
    int ncol = 0;
    for (size_t i = 0; i < n; ++i) {
        const Mesh& p = *parts[i];
        vo[i + 1] = vo[i] + p.nv;
        fo[i + 1] = fo[i] + p.nf;
        eo[i + 1] = eo[i] + p.ne;
        to[i + 1] = to[i] + p.n_patches;
        ho[i + 1] = ho[i] + (int64_t)p.halo_idx.n;
        lo[i + 1] = lo[i] + (int64_t)p.lnb.n;
        co[i + 1] = co[i] + std::max(1, p.n_comp);
        ko[i + 1] = ko[i] + (int64_t)p.col.n;
        ao[i + 1] = ao[i] + (int64_t)p.tile_adj.n;
        ceo[i + 1] = ceo[i] + (int64_t)p.cyc_e_edge.size();
        cfo[i + 1] = cfo[i] + (int64_t)p.cyc_f_face.size();
        ncol = std::max(ncol, (int)p.color_ptr_host.size() - 1);
    }
    const int64_t NV = vo[n], NF = fo[n], NE = eo[n], NT = to[n];
    if (ko[n] > INT32_MAX || 3 * NF > INT32_MAX || lo[n] > INT32_MAX || ho[n] > INT32_MAX)
        throw Error{HG_E_INVALID_ARG, "batch too large for 32-bit indices"};

    auto u = std::make_unique<Mesh>();
    Mesh& m = *u;
    m.device = p0.device;
    m.nv = NV;
    m.nf = NF;
    m.ne = NE;
    m.intrinsic = p0.intrinsic;
    m.patch_size = p0.patch_size;
    m.n_patches = (int)NT;
    double hsum = 0.0;
    for (const Mesh* p : parts) {
        m.nbnd += p->nbnd;
        m.total_area += p->total_area;
        m.max_valence = std::max(m.max_valence, p->max_valence);
        m.max_halo = std::max(m.max_halo, p->max_halo);
        m.max_ell_width = std::max(m.max_ell_width, p->max_ell_width);
        hsum += p->hbar * (double)p->ne;
        m.n_comp += std::max(1, p->n_comp);
        m.n_cycles += p->n_cycles;
        m.n_flips += p->n_flips;
        m.n_nondelaunay += p->n_nondelaunay;
    }
    m.hbar = NE > 0 ? hsum / (double)NE : 0.0;

    m.px.alloc(NV);
    m.py.alloc(NV);
    m.pz.alloc(NV);
    m.perm_v.alloc(NV);
    m.perm_f.alloc(NF);
    m.perm_e.alloc(NE);
    m.row_ptr.alloc(NV + 1);
    m.col.alloc(ko[n]);
    m.csr_edge.alloc(ko[n]);
    m.theta.alloc(ko[n]);
    m.Av.alloc(NV);
    m.sum_theta.alloc(NV);
    m.tri.alloc(3 * NF);
    m.fslot.alloc(3 * NF);
    m.fsign.alloc(NF);
    m.farea.alloc(NF);
    m.ev.alloc(2 * NE);
    m.ef.alloc(2 * NE);
    m.twin.alloc(3 * NF);
    m.h01.alloc(2 * NE);
    m.tile_ptr.alloc(NT + 1);
    m.tile_k0.alloc(NT + 1);
    m.tile_adj_ptr.alloc(NT + 1);
    m.tile_adj.alloc(ao[n]);
    m.halo_ptr.alloc(NT + 1);
    m.halo_idx.alloc(ho[n]);
    m.ell_ptr.alloc(NT + 1);
    m.lnb.alloc(lo[n]);
    m.ell_width.alloc(NT);
    m.tile_order.alloc(NT);
    m.comp_v.alloc(NV);
    m.tile_comp.alloc(NT);
    if (m.intrinsic) m.floc.alloc(3 * NF);

    for (size_t i = 0; i < n; ++i) {
        const Mesh& p = *parts[i];
        const size_t nv = p.nv, nf = p.nf, ne = p.ne, nt = p.n_patches;
        copy_into(m.px, vo[i], p.px, nv, s);
        copy_into(m.py, vo[i], p.py, nv, s);
        copy_into(m.pz, vo[i], p.pz, nv, s);
        copy_into(m.Av, vo[i], p.Av, nv, s);
        copy_into(m.sum_theta, vo[i], p.sum_theta, nv, s);
        copy_into(m.theta, ko[i], p.theta, p.col.n, s);
        copy_into(m.fsign, fo[i], p.fsign, nf, s);
        copy_into(m.farea, fo[i], p.farea, nf, s);
        copy_into(m.lnb, lo[i], p.lnb, p.lnb.n, s);
        copy_into(m.ell_width, to[i], p.ell_width, nt, s);
        if (m.intrinsic) copy_into(m.floc, 3 * fo[i], p.floc, 3 * nf, s);
        shift_into(m.perm_v.p, vo[i], p.perm_v.p, nv, vo[i], false, s);
        shift_into(m.perm_f.p, fo[i], p.perm_f.p, nf, fo[i], false, s);
        shift_into(m.perm_e.p, eo[i], p.perm_e.p, ne, eo[i], false, s);
        shift_into(m.row_ptr.p, vo[i], p.row_ptr.p, nv, ko[i], false, s);
        shift_into(m.col.p, ko[i], p.col.p, p.col.n, vo[i], false, s);
        shift_into(m.csr_edge.p, ko[i], p.csr_edge.p, p.col.n, eo[i], false, s);
        shift_into(m.tri.p, 3 * fo[i], p.tri.p, 3 * nf, vo[i], false, s);
        // slot codes (edge << 2 | flags): shift the edge field
        shift_into(reinterpret_cast<int32_t*>(m.fslot.p), 3 * fo[i], reinterpret_cast<const int32_t*>(p.fslot.p),
                   3 * nf, eo[i] * 4, false, s);
        shift_into(m.ev.p, 2 * eo[i], p.ev.p, 2 * ne, vo[i], false, s);
        shift_into(m.ef.p, 2 * eo[i], p.ef.p, 2 * ne, fo[i], true, s);
        shift_into(m.twin.p, 3 * fo[i], p.twin.p, 3 * nf, 3 * fo[i], true, s);
        shift_into(m.h01.p, 2 * eo[i], p.h01.p, 2 * ne, 3 * fo[i], true, s);
        shift_into(m.tile_ptr.p, to[i], p.tile_ptr.p, nt, vo[i], false, s);
        shift_into(m.tile_k0.p, to[i], p.tile_k0.p, nt, ko[i], false, s);
        shift_into(m.tile_adj_ptr.p, to[i], p.tile_adj_ptr.p, nt, ao[i], false, s);
        shift_into(m.tile_adj.p, ao[i], p.tile_adj.p, p.tile_adj.n, to[i], false, s);
        shift_into(m.halo_ptr.p, to[i], p.halo_ptr.p, nt, ho[i], false, s);
        shift_into(m.halo_idx.p, ho[i], p.halo_idx.p, p.halo_idx.n, vo[i], false, s);
        shift_into(m.ell_ptr.p, to[i], p.ell_ptr.p, nt, lo[i], false, s);
        shift_into(m.comp_v.p, vo[i], p.comp_v.p, nv, co[i], false, s);
        shift_into(m.tile_comp.p, to[i], p.tile_comp.p, nt, co[i], false, s);
    }
    // closing entries of the pointer arrays
    {
        const int32_t tail[5] = {(int32_t)ko[n], (int32_t)NV, (int32_t)ho[n], (int32_t)lo[n], (int32_t)ao[n]};
        HG_CHECK_HIP(hipMemcpyAsync(m.row_ptr.p + NV, &tail[0], 4, hipMemcpyHostToDevice, s));
        HG_CHECK_HIP(hipMemcpyAsync(m.tile_ptr.p + NT, &tail[1], 4, hipMemcpyHostToDevice, s));
        HG_CHECK_HIP(hipMemcpyAsync(m.tile_k0.p + NT, &tail[0], 4, hipMemcpyHostToDevice, s));
        HG_CHECK_HIP(hipMemcpyAsync(m.tile_adj_ptr.p + NT, &tail[4], 4, hipMemcpyHostToDevice, s));
        HG_CHECK_HIP(hipMemcpyAsync(m.halo_ptr.p + NT, &tail[2], 4, hipMemcpyHostToDevice, s));
        HG_CHECK_HIP(hipMemcpyAsync(m.ell_ptr.p + NT, &tail[3], 4, hipMemcpyHostToDevice, s));
        HG_CHECK_HIP(hipStreamSynchronize(s));   // tail lives on this stack frame
    }
    // colour c of the join: colour c of every member, members in order
    m.color_ptr_host.assign(ncol + 1, 0);
    {
        int64_t at = 0;
        for (int c = 0; c < ncol; ++c) {
            for (size_t i = 0; i < n; ++i) {
                const Mesh& p = *parts[i];
                if (c + 1 >= (int)p.color_ptr_host.size()) continue;
                const int c0 = p.color_ptr_host[c], cnt = p.color_ptr_host[c + 1] - c0;
                shift_into(m.tile_order.p, at, p.tile_order.p + c0, cnt, to[i], false, s);
                at += cnt;
            }
            m.color_ptr_host[c + 1] = (int32_t)at;
        }
        if (at != NT) throw Error{HG_E_DEVICE, "join: tile colours do not cover the tiles"};
    }
    // host copies
    m.iperm_v_host.resize(NV);
    for (size_t i = 0; i < n; ++i) {
        const Mesh& p = *parts[i];
        for (int64_t v = 0; v < p.nv; ++v) m.iperm_v_host[vo[i] + v] = p.iperm_v_host[v] + (int32_t)vo[i];
        // every component of a member diffuses with the member's own
        // t = m hbar^2, as the member does alone
        for (int c = 0; c < std::max(1, p.n_comp); ++c) m.comp_hbar_host.push_back(p.hbar);
    }
    // generator loops: slot pointers, edges and faces shifted
    m.cyc_e_ptr.push_back(0);
    m.cyc_f_ptr.push_back(0);
    for (size_t i = 0; i < n; ++i) {
        const Mesh& p = *parts[i];
        for (size_t k = 1; k < p.cyc_e_ptr.size(); ++k) m.cyc_e_ptr.push_back(p.cyc_e_ptr[k] + (int32_t)ceo[i]);
        for (size_t k = 1; k < p.cyc_f_ptr.size(); ++k) m.cyc_f_ptr.push_back(p.cyc_f_ptr[k] + (int32_t)cfo[i]);
        for (int32_t x : p.cyc_e_edge) m.cyc_e_edge.push_back(x + (int32_t)eo[i]);
        for (int32_t x : p.cyc_e_face) m.cyc_e_face.push_back(x + (int32_t)fo[i]);
        for (int32_t x : p.cyc_e_canon) m.cyc_e_canon.push_back(x + (int32_t)eo[i]);
        for (int32_t x : p.cyc_f_face) m.cyc_f_face.push_back(x + (int32_t)fo[i]);
        for (int32_t x : p.cyc_f_edge) m.cyc_f_edge.push_back(x + (int32_t)eo[i]);
        for (int32_t x : p.cyc_f_caller) m.cyc_f_caller.push_back(x + (int32_t)fo[i]);
        m.cyc_e_sign.insert(m.cyc_e_sign.end(), p.cyc_e_sign.begin(), p.cyc_e_sign.end());
        m.cyc_f_vec.insert(m.cyc_f_vec.end(), p.cyc_f_vec.begin(), p.cyc_f_vec.end());
    }
    m.w.ensure_pinned();
    HG_CHECK_HIP(hipStreamSynchronize(s));
    return u;
}

}  // namespace hg

namespace hg {

// The join of the most recent batch, kept for the next batch over the same
// meshes in the same order; dropped when one of them is destroyed.
struct JoinCache {
    std::mutex mu;
    std::vector<Mesh*> key;
    std::unique_ptr<Mesh> join;
    DBuf<float> d;   // the join's distances, caller order
};
static JoinCache& join_cache() {
    static JoinCache c;
    return c;
}

void forget_joins_with(Mesh* m) {
    JoinCache& c = join_cache();
    std::lock_guard<std::mutex> lock(c.mu);
    if (std::find(c.key.begin(), c.key.end(), m) != c.key.end()) {
        c.join.reset();
        c.key.clear();
        c.d.release();
    }
}

}  // namespace hg

using namespace hg;

extern "C" hg_status hg_geodesic_solve_batch(const hg_mesh_t* meshes, int32_t nq, const int32_t* const* src,
                                             const int32_t* nsrc, double t, const hg_opts* opts, float* const* d_dev,
                                             void* stream, hg_info* info) {
    return guarded([&]() -> hg_status {
        if (!meshes || !src || !nsrc || !d_dev || nq <= 0) return fail(HG_E_INVALID_ARG, "null argument or nq <= 0");
        std::vector<Mesh*> parts((size_t)nq);
        int64_t total_src = 0;
        for (int32_t i = 0; i < nq; ++i) {
            parts[i] = reinterpret_cast<Mesh*>(meshes[i]);
            if (!parts[i] || !d_dev[i] || !src[i] || nsrc[i] <= 0)
                return fail(HG_E_INVALID_ARG, "batch query " + std::to_string(i) + ": null mesh, output or sources");
            for (int32_t k = 0; k < nsrc[i]; ++k)
                if (src[i][k] < 0 || src[i][k] >= parts[i]->nv)
                    return fail(HG_E_INVALID_ARG, "batch query " + std::to_string(i) + ": source out of range");
            total_src += nsrc[i];
        }
        if (total_src > INT32_MAX) return fail(HG_E_INVALID_ARG, "too many sources");
        hipStream_t s = (hipStream_t)stream;
        JoinCache& c = join_cache();
        std::lock_guard<std::mutex> lock(c.mu);
        if (!c.join || c.key != parts) {
            c.join.reset();
            c.key.clear();
            c.d.release();
            c.join = join_meshes(parts, s);
            c.key = parts;
        }
        Mesh& J = *c.join;
        c.d.alloc((size_t)J.nv);
        // sources in the join's caller ids
        std::vector<int32_t> js;
        js.reserve((size_t)total_src);
        int64_t off = 0;
        for (int32_t i = 0; i < nq; ++i) {
            for (int32_t k = 0; k < nsrc[i]; ++k) js.push_back((int32_t)(src[i][k] + off));
            off += parts[i]->nv;
        }
        hg_opts o;
        hg_opts_default(&o);
        if (opts) o = *opts;
        o.t_per_component = 1;
        QueryOutcome q = solve_query(J, J.w, js.data(), (int32_t)js.size(), t, &o, c.d.p, s, info);
        off = 0;
        for (int32_t i = 0; i < nq; ++i) {
            HG_CHECK_HIP(hipMemcpyAsync(d_dev[i], c.d.p + off, (size_t)parts[i]->nv * sizeof(float),
                                        hipMemcpyDeviceToDevice, s));
            off += parts[i]->nv;
        }
        HG_CHECK_HIP(hipStreamSynchronize(s));
        return q.status == HG_OK ? HG_OK : fail(q.status, q.msg);
    });
}
