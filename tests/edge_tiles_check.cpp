// Host check of the face tiles of the blocked edge-ADMM launch, against a
// brute-force construction.  Linked against libhgeo.so; runs without a GPU.
//
// usage: edge_tiles_check <mesh.bin> <rings> <max_region>
//   mesh.bin: int64 nv, int64 nf, double xyz[3 nv], int32 tri[3 nf]
// Builds the library's host topology (1024-vertex tiles, as mesh creation
// does) and its face tiles, then checks, tile by tile:
//   * the tiles' faces partition [0, nf) in order, and each face's smallest
//     vertex lies in its tile's vertex range;
//   * the region is exactly the set of faces within `rings` steps of the
//     tile over shared edges (a breadth-first search written here), the
//     tile's faces first, then each ring in order of distance;
//   * every record: slot k's code is kTwinNone on a boundary slot, the
//     region-local copy 3 r' + k' of the twin when the twin's face is in
//     the region, kTwinOut otherwise; bits 48..50 are the face's signs;
//   * no face closer than `rings` steps has a twin outside the region.
// Prints "OK tiles max_region", "DOES_NOT_FIT" when the builder refuses (a
// region above max_region), or "FAIL ..." with a nonzero exit status.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <vector>

#include "../paper_1812_06060_amd/csrc/hgeo_internal.h"

static int fail(const char* what, long a, long b) {
    std::printf("FAIL %s %ld %ld\n", what, a, b);
    return 1;
}

int main(int argc, char** argv) {
    if (argc != 4) {
        std::fprintf(stderr, "usage: %s mesh.bin rings max_region\n", argv[0]);
        return 2;
    }
    const int rings = std::atoi(argv[2]), max_region = std::atoi(argv[3]);
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
    hg::build_topology(xyz.data(), nv, tri.data(), nf, 1024, T);
    hg::EdgeTiles E;
    if (!hg::build_edge_tiles(T.nf, T.tri, T.twin, T.fsign, T.tile_ptr, rings, max_region, E)) {
        std::printf("DOES_NOT_FIT\n");
        return 0;
    }
    const int nt = (int)T.tile_ptr.size() - 1;
    if ((int)E.f0.size() != nt + 1 || E.f0[0] != 0 || E.f0[nt] != T.nf) return fail("f0 range", nt, T.nf);
    if ((int64_t)E.rec.size() != E.rptr[nt] || (int64_t)E.halo.size() != E.rptr[nt] - T.nf)
        return fail("sizes", (long)E.rec.size(), (long)E.halo.size());
    std::vector<int> dist(T.nf, -1);
    int max_seen = 0;
    for (int p = 0; p < nt; ++p) {
        const int a = E.f0[p], nint = E.f0[p + 1] - a;
        if (nint < 0) return fail("tile order", p, nint);
        for (int f = a; f < a + nint; ++f) {
            int mv = std::min(T.tri[3 * f], std::min(T.tri[3 * f + 1], T.tri[3 * f + 2]));
            if (mv < T.tile_ptr[p] || mv >= T.tile_ptr[p + 1]) return fail("face tile", p, f);
        }
        // brute force: faces within `rings` steps, ring by ring
        std::vector<int> bf;
        for (int f = a; f < a + nint; ++f) {
            dist[f] = 0;
            bf.push_back(f);
        }
        size_t lo = 0;
        for (int d = 1; d <= rings; ++d) {
            const size_t hi = bf.size();
            for (size_t i = lo; i < hi; ++i)
                for (int k = 0; k < 3; ++k) {
                    const int t = T.twin[3 * (size_t)bf[i] + k];
                    if (t < 0 || dist[t / 3] >= 0) continue;
                    dist[t / 3] = d;
                    bf.push_back(t / 3);
                }
            lo = hi;
        }
        const int rb = E.rptr[p], nreg = E.rptr[p + 1] - rb;
        if (nint == 0 && nreg != 0) return fail("empty tile region", p, nreg);
        if (nreg != (int)bf.size()) return fail("region size", p, nreg - (long)bf.size());
        max_seen = std::max(max_seen, nreg);
        std::map<int, int> local;   // face -> region index
        int prev_d = 0;
        for (int r = 0; r < nreg; ++r) {
            const int x = r < nint ? a + r : E.halo[rb - a + r - nint];
            if (x < 0 || x >= T.nf || dist[x] < 0) return fail("region face", p, x);
            if ((r < nint) != (dist[x] == 0) || dist[x] < prev_d) return fail("ring order", p, r);
            prev_d = dist[x];
            if (!local.emplace(x, r).second) return fail("duplicate face", p, x);
        }
        for (int r = 0; r < nreg; ++r) {
            const int x = r < nint ? a + r : E.halo[rb - a + r - nint];
            const uint64_t w = E.rec[rb + r];
            if ((uint32_t)(w >> 48) != (uint32_t)(T.fsign[x] & 7u)) return fail("signs", p, x);
            for (int k = 0; k < 3; ++k) {
                const uint32_t code = (uint32_t)(w >> (16 * k)) & 0xFFFFu;
                const int t = T.twin[3 * (size_t)x + k];
                uint32_t want = hg::kTwinNone;
                if (t >= 0) {
                    auto it = local.find(t / 3);
                    want = it == local.end() ? hg::kTwinOut : (uint32_t)(3 * it->second + t % 3);
                }
                if (code != want) return fail("record", x, k);
                if (code == hg::kTwinOut && dist[x] < rings) return fail("twin outside too early", x, dist[x]);
            }
        }
        for (int f : bf) dist[f] = -1;
    }
    if (max_seen != E.max_region) return fail("max_region", max_seen, E.max_region);
    std::printf("OK %d %d\n", nt, E.max_region);
    return 0;
}
