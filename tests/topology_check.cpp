// Host check of the mesh topology that mesh creation builds (build_topology),
// against plain restatements of what each array must hold.  Linked against
// libhgeo.so; runs without a GPU.  The number of host worker threads is set by
// HG_HOST_THREADS, so runs with different counts can be compared by digest.
//
// usage: topology_check <mesh.bin>
//   mesh.bin: int64 nv, int64 nf, double xyz[3 nv], int32 tri[3 nf]
// Checks:
//   * perm_v / iperm_v are inverse permutations; positions follow perm_v;
//   * tiles are contiguous, at most 1024 vertices, and connected (where
//     each tile starts is not checked: comparing digests across thread
//     counts pins the whole layout);
//   * faces: tri is the caller's face perm_f[f] renumbered; the smallest
//     vertex of the faces is non-decreasing, and perm_f ascends among equal
//     smallest vertices;
//   * edges: every face slot names an edge whose endpoints are the slot's
//     endpoints and whose incident face on that side is the face; each
//     undirected mesh edge appears exactly once; the tail is the endpoint of
//     smaller caller id; the sign bit is set exactly when the slot runs from
//     tail to head; twins pair the two slots of an interior edge;
//   * perm_e orders edges by (smaller caller id, larger caller id);
//   * CSR rows list each vertex's neighbours once, ascending, with their edge;
//   * each tile's halo is the sorted set of its outside neighbours, and the
//     ELL slots map every neighbour to its local slot.
// Prints "OK <digest>" or "ERROR <code> <message>" (a refused mesh), or
// "FAIL <what> <a> <b>" with a nonzero exit status.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <set>
#include <vector>

#include "../paper_1812_06060_amd/csrc/hgeo_internal.h"

static int fail(const char* what, long a, long b) {
    std::printf("FAIL %s %ld %ld\n", what, a, b);
    return 1;
}

int main(int argc, char** argv) {
    if (argc != 2) return fail("usage", argc, 0);
    FILE* fp = std::fopen(argv[1], "rb");
    if (!fp) return fail("open", 0, 0);
    int64_t hdr[2];
    if (std::fread(hdr, sizeof(int64_t), 2, fp) != 2) return fail("read", 0, 0);
    const int64_t nv = hdr[0], nf = hdr[1];
    std::vector<double> xyz(3 * nv);
    std::vector<int32_t> tri(3 * nf);
    if (std::fread(xyz.data(), sizeof(double), xyz.size(), fp) != xyz.size()) return fail("read", 1, 0);
    if (std::fread(tri.data(), sizeof(int32_t), tri.size(), fp) != tri.size()) return fail("read", 2, 0);
    std::fclose(fp);

    hg::HostTopo T;
    try {
        hg::build_topology(xyz.data(), nv, tri.data(), nf, 1024, T, 512);
        hg::build_cycles(T);
    } catch (const hg::Error& e) {
        std::printf("ERROR %d %s\n", (int)e.code, e.msg.c_str());
        return 0;
    }
    const int64_t ne = T.ne;
    // permutations and positions
    for (int64_t i = 0; i < nv; ++i) {
        const int32_t u = T.perm_v[i];
        if (u < 0 || u >= nv || T.iperm_v[u] != i) return fail("perm_v", i, u);
        if (T.px[i] != xyz[3 * u] || T.py[i] != xyz[3 * u + 1] || T.pz[i] != xyz[3 * u + 2])
            return fail("position", i, u);
    }
    // tiles: contiguous, bounded, connected
    const int64_t np = (int64_t)T.tile_ptr.size() - 1;
    if (T.tile_ptr[0] != 0 || T.tile_ptr[np] != nv) return fail("tile_ptr ends", 0, np);
    for (int64_t p = 0; p < np; ++p) {
        const int32_t v0 = T.tile_ptr[p], v1 = T.tile_ptr[p + 1];
        if (v1 <= v0 || v1 - v0 > 1024) return fail("tile size", p, v1 - v0);
        std::vector<char> seen(v1 - v0, 0);
        std::vector<int32_t> st{v0};
        seen[0] = 1;
        int64_t n = 1;
        while (!st.empty()) {
            const int32_t x = st.back();
            st.pop_back();
            for (int32_t k = T.row_ptr[x]; k < T.row_ptr[x + 1]; ++k) {
                const int32_t y = T.col[k];
                if (y >= v0 && y < v1 && !seen[y - v0]) {
                    seen[y - v0] = 1;
                    ++n;
                    st.push_back(y);
                }
            }
        }
        if (n != v1 - v0) return fail("tile not connected", p, n);
    }
    // faces
    int32_t prev_min = -1, prev_f = -1;
    for (int64_t f = 0; f < nf; ++f) {
        const int32_t u = T.perm_f[f];
        int32_t mn = 0x7fffffff;
        for (int k = 0; k < 3; ++k) {
            if (T.tri[3 * f + k] != T.iperm_v[tri[3 * u + k]]) return fail("tri", f, k);
            mn = std::min(mn, T.tri[3 * f + k]);
        }
        if (mn < prev_min || (mn == prev_min && u <= prev_f)) return fail("face order", f, mn);
        prev_min = mn;
        prev_f = u;
    }
    // edges, slots, signs, twins
    std::map<std::pair<int32_t, int32_t>, int32_t> edge_of;
    for (int64_t e = 0; e < ne; ++e) {
        const int32_t a = T.ev[2 * e], b = T.ev[2 * e + 1];
        if (T.perm_v[a] >= T.perm_v[b]) return fail("tail", e, a);
        if (!edge_of.emplace(std::make_pair(std::min(a, b), std::max(a, b)), (int32_t)e).second)
            return fail("duplicate edge", e, a);
    }
    std::vector<int> uses(ne, 0);
    int64_t nbnd = 0;
    for (int64_t h = 0; h < 3 * nf; ++h) {
        const int64_t f = h / 3, k = h % 3;
        const int32_t a = T.tri[h], b = T.tri[3 * f + (k + 1) % 3];
        auto it = edge_of.find({std::min(a, b), std::max(a, b)});
        if (it == edge_of.end()) return fail("slot edge missing", h, 0);
        const int32_t e = it->second;
        const uint32_t sl = T.fslot[h];
        if ((int32_t)(sl >> 2) != e) return fail("fslot edge", h, e);
        const int s = (int)(sl & 1u);
        if (T.ef[2 * e + s] != f) return fail("ef", h, e);
        if (T.h01[2 * e + s] != h) return fail("h01", h, e);
        const bool bnd = T.ef[2 * e + 1] < 0;
        if ((((sl >> 1) & 1u) != 0u) != bnd) return fail("boundary bit", h, e);
        const bool plus = a == T.ev[2 * e];
        if ((((T.fsign[f] >> k) & 1) != 0) != plus) return fail("sign", h, e);
        const int32_t tw = T.h01[2 * e + 1 - s];
        if (T.twin[h] != (bnd ? -1 : tw)) return fail("twin", h, T.twin[h]);
        uses[e]++;
    }
    for (int64_t e = 0; e < ne; ++e) {
        if (uses[e] != (T.ef[2 * e + 1] < 0 ? 1 : 2)) return fail("edge use", e, uses[e]);
        nbnd += T.ef[2 * e + 1] < 0;
    }
    if (nbnd != T.nbnd) return fail("nbnd", nbnd, T.nbnd);
    // canonical edge order
    std::vector<std::pair<std::pair<int32_t, int32_t>, int32_t>> canon(ne);
    for (int64_t e = 0; e < ne; ++e) {
        const int32_t a = T.perm_v[T.ev[2 * e]], b = T.perm_v[T.ev[2 * e + 1]];
        canon[e] = {{std::min(a, b), std::max(a, b)}, (int32_t)e};
    }
    std::sort(canon.begin(), canon.end());
    for (int64_t r = 0; r < ne; ++r)
        if (T.perm_e[canon[r].second] != r) return fail("perm_e", r, canon[r].second);
    // CSR
    int maxdeg = 0;
    for (int64_t v = 0; v < nv; ++v) {
        std::set<int32_t> nb;
        for (int32_t k = T.row_ptr[v]; k < T.row_ptr[v + 1]; ++k) {
            const int32_t u = T.col[k];
            if (k > T.row_ptr[v] && T.col[k - 1] >= u) return fail("row order", v, k);
            auto it = edge_of.find({std::min<int32_t>(v, u), std::max<int32_t>(v, u)});
            if (it == edge_of.end() || it->second != T.csr_edge[k]) return fail("csr edge", v, k);
            nb.insert(u);
        }
        maxdeg = std::max<int>(maxdeg, (int)nb.size());
    }
    if ((int64_t)T.row_ptr[nv] != 2 * ne || maxdeg != T.max_valence) return fail("csr size", T.row_ptr[nv], maxdeg);
    // halos and ELL slots
    for (int64_t p = 0; p < np; ++p) {
        const int32_t v0 = T.tile_ptr[p], v1 = T.tile_ptr[p + 1];
        std::set<int32_t> out;
        int width = 0;
        for (int32_t v = v0; v < v1; ++v) {
            width = std::max(width, T.row_ptr[v + 1] - T.row_ptr[v]);
            for (int32_t k = T.row_ptr[v]; k < T.row_ptr[v + 1]; ++k)
                if (T.col[k] < v0 || T.col[k] >= v1) out.insert(T.col[k]);
        }
        std::vector<int32_t> halo(out.begin(), out.end());
        if ((int64_t)halo.size() != T.halo_ptr[p + 1] - T.halo_ptr[p]) return fail("halo size", p, halo.size());
        for (size_t j = 0; j < halo.size(); ++j)
            if (T.halo_idx[T.halo_ptr[p] + j] != halo[j]) return fail("halo", p, j);
        if (T.ell_width[p] != width) return fail("ell width", p, width);
        for (int32_t v = v0; v < v1; ++v)
            for (int32_t k = T.row_ptr[v], s = 0; k < T.row_ptr[v + 1]; ++k, ++s) {
                const int32_t u = T.col[k];
                const int l = T.lnb[T.ell_ptr[p] + (int64_t)s * 1024 + (v - v0)];
                if (l >= 1024 + (int)halo.size()) return fail("ell slot range", p, l);
                const int32_t g = l < 1024 ? v0 + l : halo[l - 1024];
                if (g != u) return fail("ell slot", p, v);
            }
    }

    // digest of every array
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void* q, size_t n) {
        const unsigned char* c = (const unsigned char*)q;
        for (size_t i = 0; i < n; ++i) {
            h ^= c[i];
            h *= 1099511628211ull;
        }
    };
#define MIXV(x) mix(x.data(), x.size() * sizeof(x[0]))
    MIXV(T.perm_v); MIXV(T.iperm_v); MIXV(T.px); MIXV(T.py); MIXV(T.pz); MIXV(T.row_ptr); MIXV(T.col);
    MIXV(T.csr_edge); MIXV(T.tri); MIXV(T.perm_f); MIXV(T.fslot); MIXV(T.fsign); MIXV(T.ev); MIXV(T.ef);
    MIXV(T.perm_e); MIXV(T.twin); MIXV(T.h01); MIXV(T.tile_ptr); MIXV(T.halo_ptr); MIXV(T.halo_idx); MIXV(T.lnb);
    MIXV(T.ell_ptr); MIXV(T.ell_width); MIXV(T.color_ptr); MIXV(T.tile_order); MIXV(T.tile_adj_ptr);
    MIXV(T.tile_adj); MIXV(T.comp); MIXV(T.tile_comp); MIXV(T.comp_hbar); MIXV(T.cyc_e_ptr); MIXV(T.cyc_e_edge);
    MIXV(T.cyc_e_face); MIXV(T.cyc_f_ptr); MIXV(T.cyc_f_face); MIXV(T.cyc_f_edge); MIXV(T.cyc_e_canon);
    MIXV(T.cyc_f_caller); MIXV(T.cyc_e_sign); MIXV(T.cyc_f_vec);
#undef MIXV
    const int64_t sc[] = {T.nv, T.nf, T.ne, T.nbnd, T.max_valence, T.patch_size, T.n_comp, T.max_halo,
                          T.max_ell_width, T.n_cycles};
    mix(sc, sizeof(sc));
    std::printf("OK %016llx\n", (unsigned long long)h);
    return 0;
}
