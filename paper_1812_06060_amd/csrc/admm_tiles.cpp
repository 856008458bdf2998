// Face tiles with halos for the blocked edge-ADMM launch (several
// iterations of the folded edge-form update, Eqs. 19-21, per launch).
//
// One iteration updates each face's three folded copies from its own copies
// and its edge-neighbours' (the twin slots), so k iterations of a face depend
// on the faces within k steps of edge adjacency.  A tile is the faces whose
// smallest internal vertex lies in one diffusion tile (a contiguous range of
// internal face ids: faces are sorted by their smallest internal vertex);
// its region is the tile followed by the faces at edge-adjacency distance
// 1, 2, ..., k from it, ring by ring.  A launch with a region resident in LDS
// runs k iterations of every region face and writes back the tile: the
// faces at distance d are exact for k - d iterations, so the tile's are exact
// after k.
//
// Per region face one 64-bit record: bits 16j..16j+15 (j = 0, 1, 2) hold the
// region-local copy index 3r + k of slot j's twin, kTwinNone for a boundary
// slot and kTwinOut for a twin outside the region; bits 48..50 hold the
// face's sign bits (Eq. 20).
#include <algorithm>

#include "hgeo_internal.h"
#include "host_par.h"

namespace hg {

namespace {

// global face id -> region-local index, open addressing, reset per tile
struct LocalMap {
    std::vector<int32_t> key, val, used;
    int mask = 0;
    explicit LocalMap(int cap_pow2) : key(cap_pow2, -1), val(cap_pow2, 0), mask(cap_pow2 - 1) {
        used.reserve(cap_pow2);
    }
    static uint32_t hash(int32_t f) { return (uint32_t)f * 2654435761u; }
    bool insert(int32_t f, int32_t r) {   // false if already present
        uint32_t h = hash(f) & mask;
        while (key[h] != -1) {
            if (key[h] == f) return false;
            h = (h + 1) & mask;
        }
        key[h] = f;
        val[h] = r;
        used.push_back((int32_t)h);
        return true;
    }
    int32_t find(int32_t f) const {
        uint32_t h = hash(f) & mask;
        while (key[h] != -1) {
            if (key[h] == f) return val[h];
            h = (h + 1) & mask;
        }
        return -1;
    }
    void clear() {
        for (int32_t h : used) key[h] = -1;
        used.clear();
    }
};

}  // namespace

bool build_edge_tiles(int64_t nf, const std::vector<int32_t>& tri, const std::vector<int32_t>& twin,
                      const std::vector<uint8_t>& fsign, const std::vector<int32_t>& tile_ptr, int rings,
                      int max_region, EdgeTiles& out) {
    const int nt = (int)tile_ptr.size() - 1;
    out = EdgeTiles{};
    out.rings = rings;
    // first face of each tile: faces are sorted by their smallest vertex
    out.f0.assign(nt + 1, 0);
    {
        int64_t f = 0;
        for (int p = 0; p < nt; ++p) {
            out.f0[p] = (int32_t)f;
            while (f < nf) {
                const int32_t mv = std::min({tri[3 * f], tri[3 * f + 1], tri[3 * f + 2]});
                if (mv >= tile_ptr[p + 1]) break;
                ++f;
            }
        }
        if (f != nf) return false;
        out.f0[nt] = (int32_t)nf;
    }
    // regions, built per tile in parallel into per-tile vectors
    std::vector<std::vector<int32_t>> halo(nt);
    std::vector<std::vector<uint64_t>> rec(nt);
    std::vector<int> nreg(nt, 0);
    const int nth = host_threads();
    std::vector<int> too_big(nth, 0);
    auto work = [&](int id) {
        int cap = 1;
        while (cap < 4 * max_region) cap <<= 1;
        LocalMap map(cap);
        std::vector<int32_t> region;
        region.reserve(2 * max_region);
        for (int p = id; p < nt; p += nth) {
            region.clear();
            map.clear();
            if (out.f0[p + 1] - out.f0[p] > max_region) {   // the map holds at most max_region faces
                too_big[id] = 1;
                return;
            }
            for (int32_t f = out.f0[p]; f < out.f0[p + 1]; ++f) {
                map.insert(f, (int32_t)region.size());
                region.push_back(f);
            }
            size_t ring0 = 0;
            bool big = false;
            for (int d = 0; d < rings && !big; ++d) {
                const size_t ring1 = region.size();
                for (size_t i = ring0; i < ring1 && !big; ++i) {
                    const int32_t x = region[i];
                    for (int k = 0; k < 3; ++k) {
                        const int32_t t = twin[3 * (size_t)x + k];
                        if (t < 0) continue;
                        const int32_t y = t / 3;
                        if (map.find(y) >= 0) continue;
                        if ((int)region.size() >= max_region) {
                            big = true;
                            break;
                        }
                        map.insert(y, (int32_t)region.size());
                        region.push_back(y);
                    }
                }
                ring0 = ring1;
            }
            if (big) {
                too_big[id] = 1;
                return;
            }
            const int nint = out.f0[p + 1] - out.f0[p];
            nreg[p] = (int)region.size();
            halo[p].assign(region.begin() + nint, region.end());
            auto& R = rec[p];
            R.resize(region.size());
            for (size_t r = 0; r < region.size(); ++r) {
                const int32_t x = region[r];
                uint64_t word = (uint64_t)(fsign[x] & 7u) << 48;
                for (int k = 0; k < 3; ++k) {
                    const int32_t t = twin[3 * (size_t)x + k];
                    uint32_t code = kTwinNone;
                    if (t >= 0) {
                        const int32_t ry = map.find(t / 3);
                        code = ry < 0 ? kTwinOut : (uint32_t)(3 * ry + t % 3);
                    }
                    word |= (uint64_t)code << (16 * k);
                }
                R[r] = word;
            }
        }
    };
    parallel_parts(nth, nth, [&](int64_t b, int64_t e, int) {
        for (int64_t id = b; id < e; ++id) work((int)id);
    });
    for (int b : too_big)
        if (b) return false;
    out.rptr.assign(nt + 1, 0);
    for (int p = 0; p < nt; ++p) {
        out.rptr[p + 1] = out.rptr[p] + nreg[p];
        out.max_region = std::max(out.max_region, nreg[p]);
    }
    const int64_t total = out.rptr[nt];
    out.rec.resize(total);
    out.halo.resize(total - nf);
    for (int p = 0; p < nt; ++p) {
        std::copy(rec[p].begin(), rec[p].end(), out.rec.begin() + out.rptr[p]);
        std::copy(halo[p].begin(), halo[p].end(), out.halo.begin() + (out.rptr[p] - out.f0[p]));
    }
    return true;
}

const Mesh::EdgeTileSet* Mesh::ensure_edge_tiles(int rings, hipStream_t s) {
    std::lock_guard<std::mutex> lock(et_mu);
    for (const auto& t : etiles)
        if (t->rings == rings) return t->ok ? t.get() : nullptr;
    auto set = std::make_unique<EdgeTileSet>();
    set->rings = rings;
    // region capacity: 3 floats per region face in LDS, at most 4 faces per
    // thread of a 1024-thread workgroup
    int lds = 0;
    HG_CHECK_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    const int cap = std::min(4096, lds / (int)(3 * sizeof(float)));
    std::vector<int32_t> tri_h((size_t)3 * nf), twin_h((size_t)3 * nf), tptr((size_t)n_patches + 1);
    std::vector<uint8_t> sign_h((size_t)nf);
    HG_CHECK_HIP(hipMemcpyAsync(tri_h.data(), tri.p, tri.bytes(), hipMemcpyDeviceToHost, s));
    HG_CHECK_HIP(hipMemcpyAsync(twin_h.data(), twin.p, twin.bytes(), hipMemcpyDeviceToHost, s));
    HG_CHECK_HIP(hipMemcpyAsync(sign_h.data(), fsign.p, fsign.bytes(), hipMemcpyDeviceToHost, s));
    HG_CHECK_HIP(hipMemcpyAsync(tptr.data(), tile_ptr.p, tile_ptr.bytes(), hipMemcpyDeviceToHost, s));
    HG_CHECK_HIP(hipStreamSynchronize(s));
    EdgeTiles T;
    if (build_edge_tiles(nf, tri_h, twin_h, sign_h, tptr, rings, cap, T)) {
        set->f0.upload(T.f0, s);
        set->rptr.upload(T.rptr, s);
        set->halo.upload(T.halo, s);
        set->rec.upload(T.rec, s);
        HG_CHECK_HIP(hipStreamSynchronize(s));   // other queries may use it once the lock is released
        set->max_region = T.max_region;
        set->n = (int)T.f0.size() - 1;
        set->ok = true;
    }
    etiles.push_back(std::move(set));
    return etiles.back()->ok ? etiles.back().get() : nullptr;
}

}  // namespace hg
