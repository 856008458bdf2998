// Edge paths between sources for the multi-source constraints of Eqs. 24-25
// (Sec. 5.2): one path from the first source of a connected component to
// each other source in it, shortest in edge count.
//
// A breadth-first tree grown from that first source alone (the same kernels
// and pairing rule as the query's breadth-first sets: parent = the neighbour
// one set closer with the smallest caller id) holds all of them: the path to
// source s has level(s) edges and is read off the parent chain.  One thread
// per path walks its chain (the only sequential part, level(s) dependent
// loads), then one thread per path slot fills in
//   edge   the internal edge id,
//   sign   +1 where the path runs along the edge's orientation halfedge
//          (smaller to larger caller id), else -1           (Eq. 25),
//   face   the face whose counter-clockwise boundary runs the edge in the
//          path's direction (the only face of a boundary edge) (Eq. 24),
//   vec    the edge vector in the path's direction          (Eq. 24).
// Sources that the tree does not reach start a new tree from the first of
// them.  The generator loops of closed components of genus > 0 (Sec. 5.1,
// built with the mesh) follow the paths as further groups of the query's
// form: edge loops with their signs (Eq. 23) or face loops with their
// polyline segments (Eq. 22).  The slots are then grouped on the host by
// edge and by face, so that the ADMM kernels can sum a group's copies in a
// fixed order.
#include <algorithm>
#include <numeric>

#include "hgeo_internal.h"

namespace hg {

constexpr int kBlockP = 256;

__global__ void k_gather_level(int n, const int32_t* idx, const int32_t* level, int32_t* out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = level[idx[i]];
}

// vert[base + L - 1 - k] = the vertex reached after k steps up from the
// source (so slots run from the root towards the source).
__global__ void k_path_walk(int np, const int32_t* src, const int32_t* base, const int32_t* len,
                            const int32_t* parent, int32_t* vert) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    int v = src[i];
    const int b = base[i], L = len[i];
    for (int k = 0; k < L; ++k) {
        vert[b + L - 1 - k] = v;
        v = parent[v];
    }
}

__global__ void k_path_slots(int ns, const int32_t* vert, const int32_t* parent, const int32_t* pedge,
                             const int32_t* ev, const int32_t* ef, const uint32_t* fslot,
                             const uint8_t* fsign, const double* px, const double* py, const double* pz,
                             int32_t* edge, float* sign, int32_t* face, float* vec) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ns) return;
    const int v = vert[k];
    const int p = parent[v];
    const int e = pedge[v];
    const bool along = ev[2 * e] == p;   // the path runs p -> v
    edge[k] = e;
    sign[k] = along ? 1.f : -1.f;
    int pick = ef[2 * e];
    for (int sd = 0; sd < 2; ++sd) {
        int f = ef[2 * e + sd];
        if (f < 0) continue;
        for (int c = 0; c < 3; ++c) {
            if (slot_edge(fslot[3 * f + c]) != e) continue;
            bool from_tail = (fsign[f] >> c) & 1;   // the face runs the edge tail -> head
            if (from_tail == along) pick = f;
        }
    }
    face[k] = pick;
    vec[3 * k] = (float)(px[v] - px[p]);
    vec[3 * k + 1] = (float)(py[v] - py[p]);
    vec[3 * k + 2] = (float)(pz[v] - pz[p]);
}

// the two face slots (3f + k) of each listed edge (-1 for a missing second face)
__global__ void k_edge_slots(int n, const int32_t* edge, const int32_t* h01, int2* out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int e = edge[i];
    out[i] = make_int2(h01[2 * e], h01[2 * e + 1]);
}

// CSR of the slots per distinct id (edge or face), slots in increasing order.
static void group_slots(const std::vector<int32_t>& id, std::vector<int32_t>& gptr, std::vector<int32_t>& gid,
                        std::vector<int32_t>& gslot) {
    const int ns = (int)id.size();
    gslot.resize(ns);
    std::iota(gslot.begin(), gslot.end(), 0);
    std::stable_sort(gslot.begin(), gslot.end(), [&](int a, int b) { return id[a] < id[b]; });
    gptr.assign(1, 0);
    gid.clear();
    for (int i = 0; i < ns; ++i) {
        if (i == 0 || id[gslot[i]] != id[gslot[i - 1]]) {
            if (i > 0) gptr.push_back(i);
            gid.push_back(id[gslot[i]]);
        }
    }
    if (ns > 0) gptr.push_back(ns);
}

void build_constraint_paths(Mesh& m, Work& w, const std::vector<int32_t>& src_internal, bool source_paths,
                            bool cycles, int form, hipStream_t s) {
    auto& P = w.paths;
    P.np = P.ns = P.max_len = 0;
    P.np_src = P.ns_src = P.n_cyc = P.ns_cyc = 0;
    std::vector<int32_t> todo;
    if (source_paths)
        for (int32_t v : src_internal)
            if (std::find(todo.begin(), todo.end(), v) == todo.end()) todo.push_back(v);
    std::vector<int32_t> h_ptr{0}, h_edge, h_face;
    std::vector<float> h_sign, h_vec;
    DBuf<int32_t> d_src, d_lvl, d_base, d_len, d_vert, d_edge, d_face;
    DBuf<float> d_sign, d_vec;
    // The sources' components: the first source of each is its root, and one
    // breadth-first search from the roots of the components holding other
    // sources gives every such component its own tree (components do not
    // touch).  The other sources are taken component by component, in order
    // of first appearance, each in the order given.
    std::vector<int32_t> rest, roots;
    if (todo.size() > 1) {
        const int nt = (int)todo.size();
        d_src.upload(todo, s);
        d_lvl.alloc(nt);
        hipLaunchKernelGGL(k_gather_level, dim3(grid_for(nt, kBlockP)), dim3(kBlockP), 0, s, nt, d_src.p, m.comp_v.p,
                           d_lvl.p);
        HG_CHECK_HIP(hipGetLastError());
        std::vector<int32_t> comp(nt);
        HG_CHECK_HIP(hipMemcpyAsync(comp.data(), d_lvl.p, nt * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HG_CHECK_HIP(hipStreamSynchronize(s));
        std::vector<int32_t> corder;   // components in order of first appearance
        std::vector<std::vector<int32_t>> members;
        for (int i = 0; i < nt; ++i) {
            const auto it = std::find(corder.begin(), corder.end(), comp[i]);
            const size_t k = (size_t)(it - corder.begin());
            if (it == corder.end()) {
                corder.push_back(comp[i]);
                members.emplace_back();
            }
            members[k].push_back(todo[i]);
        }
        for (const auto& mb : members)
            if (mb.size() > 1) {
                roots.push_back(mb[0]);
                rest.insert(rest.end(), mb.begin() + 1, mb.end());
            }
    }
    if (!rest.empty()) {
        run_bfs(m, w, roots, s);
        const int n = (int)rest.size();
        d_src.upload(rest, s);
        d_lvl.alloc(n);
        hipLaunchKernelGGL(k_gather_level, dim3(grid_for(n, kBlockP)), dim3(kBlockP), 0, s, n, d_src.p,
                           w.level.p, d_lvl.p);
        HG_CHECK_HIP(hipGetLastError());
        std::vector<int32_t> lvl(n);
        HG_CHECK_HIP(hipMemcpyAsync(lvl.data(), d_lvl.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HG_CHECK_HIP(hipStreamSynchronize(s));
        std::vector<int32_t> reached, base, len, unreached;
        int ns = 0;
        for (int i = 0; i < n; ++i) {
            if (lvl[i] < 0) {
                unreached.push_back(rest[i]);
            } else if (lvl[i] > 0) {
                reached.push_back(rest[i]);
                base.push_back(ns);
                len.push_back(lvl[i]);
                ns += lvl[i];
            }
        }
        const int np = (int)reached.size();
        if (np > 0) {
            d_src.upload(reached, s);
            d_base.upload(base, s);
            d_len.upload(len, s);
            d_vert.alloc(ns);
            d_edge.alloc(ns);
            d_face.alloc(ns);
            d_sign.alloc(ns);
            d_vec.alloc((size_t)3 * ns);
            hipLaunchKernelGGL(k_path_walk, dim3(grid_for(np, 64)), dim3(64), 0, s, np, d_src.p, d_base.p, d_len.p,
                               w.parent.p, d_vert.p);
            hipLaunchKernelGGL(k_path_slots, dim3(grid_for(ns, kBlockP)), dim3(kBlockP), 0, s, ns, d_vert.p,
                               w.parent.p, w.pedge.p, m.ev.p, m.ef.p, m.fslot.p, m.fsign.p,
                               m.px.p, m.py.p, m.pz.p, d_edge.p, d_sign.p, d_face.p, d_vec.p);
            HG_CHECK_HIP(hipGetLastError());
            const size_t o = h_edge.size();
            h_edge.resize(o + ns);
            h_face.resize(o + ns);
            h_sign.resize(o + ns);
            h_vec.resize(3 * (o + ns));
            HG_CHECK_HIP(hipMemcpyAsync(h_edge.data() + o, d_edge.p, ns * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HG_CHECK_HIP(hipMemcpyAsync(h_face.data() + o, d_face.p, ns * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HG_CHECK_HIP(hipMemcpyAsync(h_sign.data() + o, d_sign.p, ns * sizeof(float), hipMemcpyDeviceToHost, s));
            HG_CHECK_HIP(
                hipMemcpyAsync(h_vec.data() + 3 * o, d_vec.p, 3 * ns * sizeof(float), hipMemcpyDeviceToHost, s));
            HG_CHECK_HIP(hipStreamSynchronize(s));
            for (int i = 0; i < np; ++i) h_ptr.push_back((int32_t)(o + base[i] + len[i]));
        }
        if (!unreached.empty()) throw Error{HG_E_DEVICE, "source path: a source not reached from its component's root"};
    }
    P.np_src = (int)h_ptr.size() - 1;
    P.ns_src = (int)h_edge.size();
    if (cycles && m.n_cycles > 0) {
        // edge form: the loop's edges and signs (face and vector unused);
        // face form: the loop's faces and segments (edge and sign unused)
        const bool ef = form == HG_FORM_EDGE;
        const auto& cptr = ef ? m.cyc_e_ptr : m.cyc_f_ptr;
        const size_t o = h_edge.size(), n = (size_t)cptr.back();
        if (ef) {
            h_edge.insert(h_edge.end(), m.cyc_e_edge.begin(), m.cyc_e_edge.end());
            h_sign.insert(h_sign.end(), m.cyc_e_sign.begin(), m.cyc_e_sign.end());
            h_face.insert(h_face.end(), m.cyc_e_face.begin(), m.cyc_e_face.end());
            h_vec.resize(3 * (o + n), 0.f);
        } else {
            h_face.insert(h_face.end(), m.cyc_f_face.begin(), m.cyc_f_face.end());
            h_vec.insert(h_vec.end(), m.cyc_f_vec.begin(), m.cyc_f_vec.end());
            h_edge.insert(h_edge.end(), m.cyc_f_edge.begin(), m.cyc_f_edge.end());
            h_sign.resize(o + n, 0.f);
        }
        for (int c = 0; c < m.n_cycles; ++c) h_ptr.push_back((int32_t)(o + cptr[c + 1]));
        P.n_cyc = m.n_cycles;
        P.ns_cyc = (int)n;
    }
    P.np = (int)h_ptr.size() - 1;
    P.ns = (int)h_edge.size();
    P.max_len = P.max_len_src = P.max_len_cyc = 0;
    for (int i = 0; i < P.np; ++i) {
        const int len = h_ptr[i + 1] - h_ptr[i];
        int& mx = i < P.np_src ? P.max_len_src : P.max_len_cyc;
        mx = std::max(mx, len);
        P.max_len = std::max(P.max_len, len);
    }
    if (P.np == 0) return;
    P.ptr.upload(h_ptr, s);
    {
        // chunks of the edge-form projection, and the group of each slot
        std::vector<int32_t> spath(P.ns), cptr(P.np + 1, 0), chunk_path;
        for (int i = 0; i < P.np; ++i) {
            for (int k = h_ptr[i]; k < h_ptr[i + 1]; ++k) spath[k] = i;
            const int nc = (h_ptr[i + 1] - h_ptr[i] + kPathChunk - 1) / kPathChunk;
            cptr[i + 1] = cptr[i] + nc;
            for (int c = 0; c < nc; ++c) chunk_path.push_back(i);
        }
        P.nch = cptr[P.np];
        P.spath.upload(spath, s);
        P.cptr.upload(cptr, s);
        P.chunk_path.upload(chunk_path, s);
        P.pc.alloc((size_t)2 * P.nch);   // edge form: one sum per chunk, face form: two
    }
    P.edge.upload(h_edge, s);
    P.face.upload(h_face, s);
    P.sign.upload(h_sign, s);
    P.vec.upload(h_vec, s);
    std::vector<int32_t> gptr, gid, gslot;
    group_slots(h_edge, gptr, gid, gslot);
    P.ng_edge = (int)gid.size();
    P.eg_ptr.upload(gptr, s);
    P.eg_id.upload(gid, s);
    P.eg_slot.upload(gslot, s);
    P.zslot.alloc(P.ns);
    hipLaunchKernelGGL(k_edge_slots, dim3(grid_for(P.ns, kBlockP)), dim3(kBlockP), 0, s, P.ns, P.edge.p, m.h01.p,
                       P.zslot.p);
    P.gzslot.alloc(P.ng_edge);
    hipLaunchKernelGGL(k_edge_slots, dim3(grid_for(P.ng_edge, kBlockP)), dim3(kBlockP), 0, s, P.ng_edge,
                       P.eg_id.p, m.h01.p, P.gzslot.p);
    HG_CHECK_HIP(hipGetLastError());
    group_slots(h_face, gptr, gid, gslot);
    P.ng_face = (int)gid.size();
    P.fg_ptr.upload(gptr, s);
    P.fg_id.upload(gid, s);
    P.fg_slot.upload(gslot, s);
    HG_CHECK_HIP(hipStreamSynchronize(s));   // host vectors go out of scope
}

}  // namespace hg
