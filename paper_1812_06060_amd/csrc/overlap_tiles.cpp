// Overlapping diffusion tiles: each tile's LDS region is its core (the tile's
// own vertices) plus `rings` rings of overlap vertices around it, which the
// in-tile sweeps update as well, plus the ring beyond them, held fixed.
// Only the core is written back.
//
// Why: with a one-ring halo, the relative error of u at a tile's side
// boundary is taken over from the neighbouring tile at the same distance
// from the sources, and such side-to-side exchange is what keeps the
// block iteration slow once the front has passed.  A few rings of overlap
// let the in-tile sweeps settle the core's sides against values that are
// themselves being relaxed (an overlapping Schwarz iteration); the fixed
// point is unchanged, since at convergence every core vertex satisfies
// Eq. 7 for the converged values around it.
//
// Layout per tile p (halo_idx[halo_ptr[p] ..]): the n_ov[p] overlap vertices
// (sorted), then the fixed outer ring (sorted).  LDS slots: core i -> i,
// overlap j -> P + j, outer ring j -> P + n_ov + j.  ELL rows: the core's
// (width x P, stride P, as for the plain tiles) followed by the overlap
// vertices' (width x n_ov, stride n_ov), neighbours in CSR order.
// Colours: a tile reads the cores of the tiles its overlap and outer ring
// reach, so two tiles get different colours whenever either one reads the
// other's core; tiles of one colour then never read what another writes.
#include <algorithm>

#include "hgeo_internal.h"

namespace hg {

bool build_overlap_tiles(const std::vector<int32_t>& row_ptr, const std::vector<int32_t>& col,
                         const std::vector<int32_t>& tile_ptr, int P, int rings, int max_ov, OverlapTiles& out,
                         size_t lds_budget, int lds_width) {
    const int64_t nv = (int64_t)row_ptr.size() - 1;
    const int64_t np = (int64_t)tile_ptr.size() - 1;
    std::vector<int32_t> tile_of(nv);
    for (int64_t p = 0; p < np; ++p)
        for (int32_t v = tile_ptr[p]; v < tile_ptr[p + 1]; ++v) tile_of[v] = (int32_t)p;
    out = OverlapTiles();
    out.rings = rings;
    out.halo_ptr.assign(np + 1, 0);
    out.n_ov.assign(np, 0);
    out.ell_ptr.assign(np + 1, 0);
    out.ell_width.assign(np, 0);
    std::vector<int32_t> ov, ring, front, next;
    std::vector<std::vector<int32_t>> reads(np);   // tiles whose core p reads
    std::vector<int32_t> tag(nv, -1);   // marks of the current attempt
    int stamp = 0;
    for (int64_t p = 0; p < np; ++p) {
        const int32_t v0 = tile_ptr[p], v1 = tile_ptr[p + 1];
        // the tile's rings: as many as requested while its region fits the
        // LDS budget and the overlap fits the threads (fewer for a tile
        // with a long boundary; the fixed point does not depend on them)
        for (int rr = rings;; --rr) {
            ++stamp;
            for (int32_t v = v0; v < v1; ++v) tag[v] = stamp;
            ov.clear();
            front.clear();
            for (int32_t v = v0; v < v1; ++v) front.push_back(v);
            for (int r = 0; r < rr; ++r) {
                next.clear();
                for (int32_t v : front)
                    for (int32_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) {
                        const int32_t u = col[k];
                        if (tag[u] != stamp) {
                            tag[u] = stamp;
                            next.push_back(u);
                        }
                    }
                ov.insert(ov.end(), next.begin(), next.end());
                front.swap(next);
            }
            ring.clear();
            for (int32_t v : front)
                for (int32_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) {
                    const int32_t u = col[k];
                    if (tag[u] != stamp) {
                        tag[u] = stamp;
                        ring.push_back(u);
                    }
                }
            const size_t need = (((size_t)(P + ov.size() + ring.size()) * 20 + 7) & ~(size_t)7) +
                                ov.size() * (size_t)lds_width * 10;
            if (((int)ov.size() <= max_ov && need <= lds_budget) || rr == 0) break;
        }
        if ((int)ov.size() > max_ov) return false;
        std::sort(ov.begin(), ov.end());
        std::sort(ring.begin(), ring.end());
        const int64_t nreg = (int64_t)P + (int64_t)ov.size() + (int64_t)ring.size();
        if (nreg >= 65535) return false;   // 16-bit local slots
        out.n_ov[p] = (int32_t)ov.size();
        out.halo_idx.insert(out.halo_idx.end(), ov.begin(), ov.end());
        out.halo_idx.insert(out.halo_idx.end(), ring.begin(), ring.end());
        out.halo_ptr[p + 1] = (int32_t)out.halo_idx.size();
        out.max_halo = std::max<int>(out.max_halo, (int)(ov.size() + ring.size()));
        out.max_ov = std::max<int>(out.max_ov, (int)ov.size());
        for (int32_t u : ov) reads[p].push_back(tile_of[u]);
        for (int32_t u : ring) reads[p].push_back(tile_of[u]);
        // ELL rows: core rows, then overlap rows
        int width = 0;
        for (int32_t v = v0; v < v1; ++v) width = std::max(width, row_ptr[v + 1] - row_ptr[v]);
        for (int32_t u : ov) width = std::max(width, row_ptr[u + 1] - row_ptr[u]);
        if (width > 255) return false;
        out.ell_width[p] = (uint8_t)width;
        out.max_ell_width = std::max(out.max_ell_width, width);
        const int64_t no = (int64_t)ov.size();
        const int64_t base = (int64_t)out.lnb.size();
        out.ell_ptr[p] = (int32_t)base;
        out.lnb.resize(base + (int64_t)width * (P + no), (uint16_t)0xFFFF);
        auto slot_of = [&](int32_t u) -> uint16_t {
            if (u >= v0 && u < v1) return (uint16_t)(u - v0);
            auto it = std::lower_bound(ov.begin(), ov.end(), u);
            if (it != ov.end() && *it == u) return (uint16_t)(P + (it - ov.begin()));
            auto jt = std::lower_bound(ring.begin(), ring.end(), u);
            return (uint16_t)(P + no + (jt - ring.begin()));
        };
        for (int32_t v = v0; v < v1; ++v) {
            int s = 0;
            for (int32_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k, ++s)
                out.lnb[base + (int64_t)s * P + (v - v0)] = slot_of(col[k]);
        }
        for (int64_t j = 0; j < no; ++j) {
            const int32_t u = ov[j];
            int s = 0;
            for (int32_t k = row_ptr[u]; k < row_ptr[u + 1]; ++k, ++s)
                out.lnb[base + (int64_t)width * P + (int64_t)s * no + j] = slot_of(col[k]);
        }
        if ((int64_t)out.lnb.size() >= (1ll << 31)) return false;
    }
    out.ell_ptr[np] = (int32_t)out.lnb.size();
    // colouring: conflict when either tile reads the other's core
    std::vector<std::vector<int32_t>> conf(np);
    for (int64_t p = 0; p < np; ++p) {
        auto& r = reads[p];
        std::sort(r.begin(), r.end());
        r.erase(std::unique(r.begin(), r.end()), r.end());
        for (int32_t q : r)
            if (q != (int32_t)p) {
                conf[p].push_back(q);
                conf[q].push_back((int32_t)p);
            }
    }
    for (auto& a : conf) {
        std::sort(a.begin(), a.end());
        a.erase(std::unique(a.begin(), a.end()), a.end());
    }
    colour_tiles(conf, out.color_ptr, out.tile_order);
    return true;
}

const Mesh::OverlapTileSet* Mesh::ensure_overlap_tiles(int rings, int max_ov, size_t lds_budget, int lds_width,
                                                       hipStream_t s) {
    std::lock_guard<std::mutex> lock(ot_mu);
    for (const auto& t : otiles)
        if (t->rings == rings) return t->ok ? t.get() : nullptr;
    auto set = std::make_unique<OverlapTileSet>();
    set->rings = rings;
    std::vector<int32_t> rp((size_t)nv + 1), cl(col.n), tp((size_t)n_patches + 1);
    HG_CHECK_HIP(hipMemcpyAsync(rp.data(), row_ptr.p, row_ptr.bytes(), hipMemcpyDeviceToHost, s));
    HG_CHECK_HIP(hipMemcpyAsync(cl.data(), col.p, col.bytes(), hipMemcpyDeviceToHost, s));
    HG_CHECK_HIP(hipMemcpyAsync(tp.data(), tile_ptr.p, tile_ptr.bytes(), hipMemcpyDeviceToHost, s));
    HG_CHECK_HIP(hipStreamSynchronize(s));
    OverlapTiles T;
    if (build_overlap_tiles(rp, cl, tp, patch_size, rings, max_ov, T, lds_budget, lds_width)) {
        set->halo_ptr.upload(T.halo_ptr, s);
        set->halo_idx.upload(T.halo_idx, s);
        set->n_ov.upload(T.n_ov, s);
        set->ell_ptr.upload(T.ell_ptr, s);
        set->ell_width.upload(T.ell_width, s);
        set->lnb.upload(T.lnb, s);
        set->tile_order.upload(T.tile_order, s);
        set->color_ptr_host = T.color_ptr;
        set->max_halo = T.max_halo;
        set->max_ov = T.max_ov;
        set->max_ell_width = T.max_ell_width;
        HG_CHECK_HIP(hipStreamSynchronize(s));   // other queries may use it once the lock is released
        set->ok = true;
    }
    otiles.push_back(std::move(set));
    return otiles.back()->ok ? otiles.back().get() : nullptr;
}

}  // namespace hg
