// Homology generators for the global integrability of closed surfaces of
// genus g > 0 (Sec. 5.1, Eqs. 22-23).
//
// Local conditions (zero curl per face in the face form, zero sum around
// every vertex-dual loop in the edge form) make a field integrable on a disk
// or a sphere, but on a torus-like component they leave 2g loops free: a
// field can circulate around the handles.  One constraint per generator loop
// (zero circulation) closes that gap; each loop is a constraint group of the
// same kind as a source path of Eqs. 24-25, so the ADMM treats both alike.
//
// The basis comes from a tree-cotree decomposition, with every choice made
// on the caller's ids so that the loops do not depend on the internal
// numbering:
//   * primal tree T: breadth-first from the smallest vertex of each
//     component, parent = the neighbour one level closer with the smallest
//     id;
//   * dual tree C: first-in-first-out breadth-first search over faces from
//     the smallest face of each component, a face's edges taken in slot
//     order (tri[k], tri[k+1]), crossing only interior edges not in T;
//   * generators: the interior edges in neither tree, in canonical edge
//     order, of components without boundary (holes of components with
//     boundary are not constrained).
// For a generator e = (a, b), a < b:
//   edge loop: a -> b along e, then back to a through T (up from b to the
//     lowest common ancestor, down to a); sign +1 where the loop runs from
//     the smaller to the larger caller id;
//   face loop: f0 -> f1 across e (f0 < f1 its faces), then back to f0
//     through C; per face the polyline segment from the midpoint of the
//     edge it is entered by to the midpoint of the edge it is left by.
// A component with Euler characteristic 2 (a sphere) has no generator, so
// the trees are only grown when some closed component has a lower one.
#include <algorithm>

#include "hgeo_internal.h"

namespace hg {

void build_cycles(HostTopo& T) {
    T.n_cycles = 0;
    T.cyc_e_ptr.assign(1, 0);
    T.cyc_f_ptr.assign(1, 0);
    T.cyc_e_edge.clear();
    T.cyc_e_sign.clear();
    T.cyc_e_face.clear();
    T.cyc_e_canon.clear();
    T.cyc_f_caller.clear();
    T.cyc_f_face.clear();
    T.cyc_f_edge.clear();
    T.cyc_f_vec.clear();
    const int64_t nv = T.nv, nf = T.nf, ne = T.ne;
    const int nc = T.n_comp;

    // Euler characteristic and boundary of each component
    std::vector<int64_t> chi(nc, 0);
    std::vector<char> open(nc, 0);
    for (int64_t v = 0; v < nv; ++v) chi[T.comp[v]] += 1;
    for (int64_t e = 0; e < ne; ++e) {
        const int c = T.comp[T.ev[2 * e]];
        chi[c] -= 1;
        if (T.ef[2 * e + 1] < 0) open[c] = 1;
    }
    for (int64_t f = 0; f < nf; ++f) chi[T.comp[T.tri[3 * f]]] += 1;
    bool any = false;
    for (int c = 0; c < nc; ++c) any = any || (!open[c] && chi[c] < 2);
    if (!any) return;

    // caller-id views
    std::vector<int32_t> iperm_f(nf);
    for (int64_t f = 0; f < nf; ++f) iperm_f[T.perm_f[f]] = (int32_t)f;
    std::vector<int32_t> iperm_e(ne);
    for (int64_t e = 0; e < ne; ++e) iperm_e[T.perm_e[e]] = (int32_t)e;
    auto edge_between = [&](int32_t a_caller, int32_t b_caller) {
        const int32_t a = T.iperm_v[a_caller], b = T.iperm_v[b_caller];
        for (int32_t k = T.row_ptr[a]; k < T.row_ptr[a + 1]; ++k)
            if (T.col[k] == b) return T.csr_edge[k];
        throw Error{HG_E_DEVICE, "cycle basis: loop steps over a missing edge"};
    };

    // primal tree: levels from the component roots, parent by smallest id
    std::vector<int32_t> level(nv, -1), parent(nv, -1), queue;
    queue.reserve(nv);
    {
        std::vector<char> has_root(nc, 0);
        for (int64_t u = 0; u < nv; ++u) {
            const int c = T.comp[T.iperm_v[u]];
            if (has_root[c]) continue;
            has_root[c] = 1;
            level[u] = 0;
            queue.push_back((int32_t)u);
        }
        for (size_t q = 0; q < queue.size(); ++q) {
            const int32_t u = queue[q], ui = T.iperm_v[u];
            for (int32_t k = T.row_ptr[ui]; k < T.row_ptr[ui + 1]; ++k) {
                const int32_t x = T.perm_v[T.col[k]];
                if (level[x] < 0) {
                    level[x] = level[u] + 1;
                    queue.push_back(x);
                }
            }
        }
    }
    std::vector<char> in_t(ne, 0), in_c(ne, 0);
    for (int64_t u = 0; u < nv; ++u) {
        if (level[u] <= 0) continue;
        const int32_t ui = T.iperm_v[u];
        int32_t best = -1, best_e = -1;
        for (int32_t k = T.row_ptr[ui]; k < T.row_ptr[ui + 1]; ++k) {
            const int32_t x = T.perm_v[T.col[k]];
            if (level[x] == level[u] - 1 && (best < 0 || x < best)) {
                best = x;
                best_e = T.csr_edge[k];
            }
        }
        parent[u] = best;
        in_t[best_e] = 1;
    }

    // dual tree over caller faces
    std::vector<int32_t> fpar(nf, -1), fpar_e(nf, -1);
    std::vector<char> seen(nf, 0);
    std::vector<int32_t> fq;
    fq.reserve(nf);
    for (int64_t f0 = 0; f0 < nf; ++f0) {
        if (seen[f0]) continue;
        seen[f0] = 1;
        fq.clear();
        fq.push_back((int32_t)f0);
        for (size_t q = 0; q < fq.size(); ++q) {
            const int32_t f = fq[q], fi = iperm_f[f];
            for (int k = 0; k < 3; ++k) {
                const uint32_t sl = T.fslot[3 * (int64_t)fi + k];
                if (slot_bnd(sl)) continue;
                const int32_t e = slot_edge(sl);
                if (in_t[e]) continue;
                const int32_t oi = T.ef[2 * e] == fi ? T.ef[2 * e + 1] : T.ef[2 * e];
                const int32_t g = T.perm_f[oi];
                if (seen[g]) continue;
                seen[g] = 1;
                fpar[g] = f;
                fpar_e[g] = e;
                in_c[e] = 1;
                fq.push_back(g);
            }
        }
    }

    // loop through a tree: b up to the lowest common ancestor c, then down
    // to a (both ends included)
    std::vector<int32_t> stamp_v(nv, -1), stamp_f(nf, -1);
    auto tree_loop = [](int32_t a, int32_t b, const std::vector<int32_t>& par, std::vector<int32_t>& stamp,
                        int32_t tag, std::vector<int32_t>& out) {
        for (int32_t x = a; x >= 0; x = par[x]) stamp[x] = tag;
        out.clear();
        int32_t c = b;
        while (stamp[c] != tag) {
            out.push_back(c);
            c = par[c];
            if (c < 0) throw Error{HG_E_DEVICE, "cycle basis: tree loop leaves its component"};
        }
        out.push_back(c);
        const size_t mid = out.size();
        for (int32_t x = a; x != c; x = par[x]) out.push_back(x);
        std::reverse(out.begin() + mid, out.end());
    };

    auto midpoint = [&](int32_t e, int c) {
        const int32_t a = T.ev[2 * e], b = T.ev[2 * e + 1];
        const double* P = c == 0 ? T.px.data() : c == 1 ? T.py.data() : T.pz.data();
        return 0.5 * (P[a] + P[b]);
    };

    std::vector<int32_t> loop, floop, cross;
    int32_t tag = 0;
    for (int64_t r = 0; r < ne; ++r) {
        const int32_t e = iperm_e[r];
        if (T.ef[2 * e + 1] < 0 || in_t[e] || in_c[e] || open[T.comp[T.ev[2 * e]]]) continue;
        // edge loop (Eq. 23)
        int32_t a = T.perm_v[T.ev[2 * e]], b = T.perm_v[T.ev[2 * e + 1]];
        if (a > b) std::swap(a, b);
        tree_loop(a, b, parent, stamp_v, tag, loop);
        loop.insert(loop.begin(), a);   // a, b, ..., c, ..., a
        for (size_t i = 0; i + 1 < loop.size(); ++i) {
            const int32_t ee = edge_between(loop[i], loop[i + 1]);
            T.cyc_e_edge.push_back(ee);
            T.cyc_e_face.push_back(T.ef[2 * ee]);
            T.cyc_e_canon.push_back(T.perm_e[ee]);
            T.cyc_e_sign.push_back(loop[i] < loop[i + 1] ? 1.f : -1.f);
        }
        T.cyc_e_ptr.push_back((int32_t)T.cyc_e_edge.size());
        // face loop (Eq. 22)
        int32_t f0 = T.perm_f[T.ef[2 * e]], f1 = T.perm_f[T.ef[2 * e + 1]];
        if (f0 > f1) std::swap(f0, f1);
        tree_loop(f0, f1, fpar, stamp_f, tag, floop);
        floop.insert(floop.begin(), f0);   // f0, f1, ..., f0
        const size_t n = floop.size() - 1;
        cross.assign(1, e);
        for (size_t i = 1; i < n; ++i) {
            const int32_t x = floop[i], y = floop[i + 1];
            cross.push_back(fpar[x] == y ? fpar_e[x] : fpar_e[y]);
        }
        for (size_t i = 0; i < n; ++i) {
            const int32_t in_e = cross[(i + n - 1) % n], out_e = cross[i];
            T.cyc_f_face.push_back(iperm_f[floop[i]]);
            T.cyc_f_caller.push_back(floop[i]);
            T.cyc_f_edge.push_back(out_e);
            for (int c = 0; c < 3; ++c) T.cyc_f_vec.push_back((float)(midpoint(out_e, c) - midpoint(in_e, c)));
        }
        T.cyc_f_ptr.push_back((int32_t)T.cyc_f_face.size());
        ++tag;
        ++T.n_cycles;
    }
}

}  // namespace hg
