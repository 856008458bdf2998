// Host check of the overlapping diffusion tiles against a brute-force
// construction.  Linked against libhgeo.so; runs without a GPU.
//
// usage: overlap_tiles_check <mesh.bin> <rings> <max_ov>
//   mesh.bin: int64 nv, int64 nf, double xyz[3 nv], int32 tri[3 nf]
// Builds the library's host topology (1024-vertex tiles, as mesh creation
// does) and its overlapping tiles, then checks, tile by tile:
//   * the overlap vertices are exactly those at hop distance 1..r from the
//     tile's core (a breadth-first search written here), sorted, and the
//     fixed ring exactly those at distance r + 1, sorted, where r = rings,
//     or fewer when rings would give the tile more than max_ov overlap
//     vertices (then r + 1 rings would, too);
//   * every ELL row (the core's, stride 1024, then the overlap vertices',
//     stride n_ov) decodes, slot by slot, to the vertex's CSR neighbours in
//     order, padding 0xFFFF after them;
//   * no tile reads (core, overlap or ring) the core of another tile of its
//     own colour, and every tile has a colour.
// Prints "OK tiles max_ov colours shrunk" (shrunk: tiles with fewer than
// `rings` rings), "DOES_NOT_FIT" when the builder refuses, or "FAIL ..."
// with a nonzero exit status.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_1812_06060_amd/csrc/hgeo_internal.h"

static int fail(const char* what, long a, long b) {
    std::printf("FAIL %s %ld %ld\n", what, a, b);
    return 1;
}

int main(int argc, char** argv) {
    if (argc != 4) {
        std::fprintf(stderr, "usage: %s mesh.bin rings max_ov\n", argv[0]);
        return 2;
    }
    const int rings = std::atoi(argv[2]), max_ov = std::atoi(argv[3]);
    FILE* fp = std::fopen(argv[1], "rb");
    if (!fp) return 2;
    int64_t nv = 0, nf = 0;
    if (std::fread(&nv, 8, 1, fp) != 1 || std::fread(&nf, 8, 1, fp) != 1) return 2;
    std::vector<double> xyz(3 * nv);
    std::vector<int32_t> tri(3 * nf);
    if (std::fread(xyz.data(), 8, xyz.size(), fp) != xyz.size()) return 2;
    if (std::fread(tri.data(), 4, tri.size(), fp) != tri.size()) return 2;
    std::fclose(fp);

    hg::HostTopo T;
    const int P = 1024;
    hg::build_topology(xyz.data(), nv, tri.data(), nf, P, T);
    hg::OverlapTiles O;
    if (!hg::build_overlap_tiles(T.row_ptr, T.col, T.tile_ptr, P, rings, max_ov, O)) {
        std::printf("DOES_NOT_FIT\n");
        return 0;
    }
    const int nt = (int)T.tile_ptr.size() - 1;
    std::vector<int> tile_of(nv), dist(nv, -1), color(nt, -1);
    for (int p = 0; p < nt; ++p)
        for (int v = T.tile_ptr[p]; v < T.tile_ptr[p + 1]; ++v) tile_of[v] = p;
    const int ncol = (int)O.color_ptr.size() - 1;
    for (int c = 0; c < ncol; ++c)
        for (int k = O.color_ptr[c]; k < O.color_ptr[c + 1]; ++k) {
            const int p = O.tile_order[k];
            if (p < 0 || p >= nt || color[p] >= 0) return fail("tile order", c, p);
            color[p] = c;
        }
    for (int p = 0; p < nt; ++p)
        if (color[p] < 0) return fail("uncoloured tile", p, 0);
    int max_seen = 0, shrunk = 0;
    for (int p = 0; p < nt; ++p) {
        const int v0 = T.tile_ptr[p], v1 = T.tile_ptr[p + 1];
        // brute force: hop distance from the core, up to rings + 2
        std::vector<int> seen;
        std::vector<int> fr;
        for (int v = v0; v < v1; ++v) {
            dist[v] = 0;
            seen.push_back(v);
            fr.push_back(v);
        }
        for (int d = 1; d <= rings + 2; ++d) {
            std::vector<int> nx;
            for (int v : fr)
                for (int k = T.row_ptr[v]; k < T.row_ptr[v + 1]; ++k) {
                    const int u = T.col[k];
                    if (dist[u] >= 0) continue;
                    dist[u] = d;
                    seen.push_back(u);
                    nx.push_back(u);
                }
            fr.swap(nx);
        }
        const int h0 = O.halo_ptr[p], nh = O.halo_ptr[p + 1] - h0, no = O.n_ov[p];
        // the rings this tile got: the largest distance among its overlap
        int r = 0;
        for (int j = 0; j < no; ++j) {
            const int u = O.halo_idx[h0 + j];
            if (u < 0 || u >= nv || dist[u] < 1) return fail("overlap vertex not near the core", p, j);
            r = std::max(r, dist[u]);
        }
        if (r > rings) return fail("too many rings", p, r);
        std::vector<int> ov, ring;
        int next_ov = 0;
        for (int u : seen) {
            if (dist[u] >= 1 && dist[u] <= r) ov.push_back(u);
            if (dist[u] == r + 1) ring.push_back(u);
            if (dist[u] >= 1 && dist[u] <= r + 1) ++next_ov;
        }
        if (r < rings && next_ov > no) {   // (a component exhausted at r needs no further rings)
            ++shrunk;
            if (next_ov <= max_ov) return fail("rings cut without need", p, r);
        }
        std::sort(ov.begin(), ov.end());
        std::sort(ring.begin(), ring.end());
        if (no != (int)ov.size()) return fail("overlap size", p, no - (long)ov.size());
        if (nh != (int)(ov.size() + ring.size())) return fail("halo size", p, nh);
        for (int j = 0; j < no; ++j)
            if (O.halo_idx[h0 + j] != ov[j]) return fail("overlap vertex", p, j);
        for (int j = 0; j < (int)ring.size(); ++j)
            if (O.halo_idx[h0 + no + j] != ring[j]) return fail("ring vertex", p, j);
        max_seen = std::max(max_seen, no);
        // decode a local slot to its vertex
        auto vertex_of = [&](int l) -> int {
            if (l < P) return v0 + l;
            return O.halo_idx[h0 + (l - P)];
        };
        const int W = O.ell_width[p], eb = O.ell_ptr[p];
        auto check_row = [&](int v, int base, int stride, int i) -> bool {
            const int deg = T.row_ptr[v + 1] - T.row_ptr[v];
            if (deg > W) return false;
            for (int s = 0; s < W; ++s) {
                const uint16_t l = O.lnb[base + s * stride + i];
                if (s < deg) {
                    if (l == 0xFFFF || l >= P + nh) return false;
                    if (vertex_of(l) != T.col[T.row_ptr[v] + s]) return false;
                } else if (l != 0xFFFF) {
                    return false;
                }
            }
            return true;
        };
        for (int v = v0; v < v1; ++v)
            if (!check_row(v, eb, P, v - v0)) return fail("core row", p, v - v0);
        for (int j = 0; j < no; ++j)
            if (!check_row(ov[j], eb + W * P, no, j)) return fail("overlap row", p, j);
        if (p + 1 < nt && O.ell_ptr[p + 1] - eb != W * (P + no)) return fail("ell block", p, O.ell_ptr[p + 1] - eb);
        // colours: no same-colour tile's core within the read region
        for (int u : seen)
            if (dist[u] >= 1 && dist[u] <= r + 1 && tile_of[u] != p && color[tile_of[u]] == color[p])
                return fail("colour", p, tile_of[u]);
        for (int u : seen) dist[u] = -1;
    }
    std::printf("OK %d %d %d %d\n", nt, max_seen, ncol, shrunk);
    return 0;
}
