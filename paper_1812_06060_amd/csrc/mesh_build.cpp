// Host-side connectivity of a triangle mesh for the hgeo library.
//
// Builds, in linear time (bucket sorts keyed by vertex id):
//   * tiles: connected patches of at most patch_size vertices, grown
//     breadth-first from seeds taken in 3D Morton order of the positions;
//     the internal vertex order is tile-major;
//   * faces sorted by their smallest internal vertex;
//   * unique edges, the orientation halfedge of each (from the smaller to the
//     larger caller vertex id, Sec. 4.1), the incident faces, and per face
//     slot the edge, the side and the integrability sign of Eq. 20;
//   * the canonical (caller-facing) edge numbering;
//   * the CSR one-ring adjacency used by the breadth-first sets (Eq. 6) and
//     the diffusion sweeps (Eq. 7);
//   * per tile: its halo (outside one-ring) and the tile-local neighbour
//     slots of every vertex (ELL layout).
// Geometry (areas, cotangent weights) is computed later on the GPU.  The
// per-element phases run on host worker threads (host_par.h); every output
// is the same for any number of them.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "hgeo_internal.h"
#include "host_par.h"

namespace hg {

static inline uint64_t spread3(uint64_t x) {
    x &= 0x1fffff;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}

static void bad(const std::string& msg) { throw Error{HG_E_BAD_MESH, msg}; }

// Items 0..n-1 grouped by key (keys[i] in [0, nk)), in increasing i within a
// key: items[ptr[k] .. ptr[k+1]) -- a stable counting sort.  Each worker owns
// a range of keys and scans all of them, so the result is the sequential one.
static void group_by_key(const std::vector<int32_t>& keys, int64_t nk, std::vector<int32_t>& ptr,
                         std::vector<int32_t>& items) {
    const int64_t n = (int64_t)keys.size();
    const int parts = host_threads();
    ptr.assign(nk + 1, 0);
    items.assign(n, 0);
    parallel_parts(nk, parts, [&](int64_t k0, int64_t k1, int) {
        for (int64_t i = 0; i < n; ++i) {
            const int32_t k = keys[i];
            if (k >= k0 && k < k1) ++ptr[k + 1];
        }
    });
    for (int64_t k = 0; k < nk; ++k) ptr[k + 1] += ptr[k];
    parallel_parts(nk, parts, [&](int64_t k0, int64_t k1, int) {
        std::vector<int32_t> pos(ptr.begin() + k0, ptr.begin() + k1);
        for (int64_t i = 0; i < n; ++i) {
            const int32_t k = keys[i];
            if (k >= k0 && k < k1) items[pos[k - k0]++] = (int32_t)i;
        }
    });
}

void build_topology(const double* xyz, int64_t nv, const int32_t* tri_in, int64_t nf,
                    int patch_size, HostTopo& T, int slots) {
    if (nv <= 0 || nf <= 0) throw Error{HG_E_INVALID_ARG, "empty mesh"};
    if (nv >= (1ll << 31) || 3 * nf >= (1ll << 31))
        throw Error{HG_E_INVALID_ARG, "mesh too large for 32-bit element indices"};
    T.nv = nv;
    T.nf = nf;
    // ---- validation of indices and degenerate faces
    for (int64_t f = 0; f < nf; ++f) {
        int32_t a = tri_in[3 * f], b = tri_in[3 * f + 1], c = tri_in[3 * f + 2];
        if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv)
            bad("triangle " + std::to_string(f) + " has a vertex index out of range");
        if (a == b || b == c || a == c) bad("triangle " + std::to_string(f) + " repeats a vertex");
    }
    for (int64_t i = 0; i < 3 * nv; ++i)
        if (!std::isfinite(xyz[i])) throw Error{HG_E_INVALID_ARG, "non-finite vertex position"};

    // ---- Morton order of the vertices
    double lo[3] = {xyz[0], xyz[1], xyz[2]}, hi[3] = {xyz[0], xyz[1], xyz[2]};
    for (int64_t i = 0; i < nv; ++i)
        for (int c = 0; c < 3; ++c) {
            lo[c] = std::min(lo[c], xyz[3 * i + c]);
            hi[c] = std::max(hi[c], xyz[3 * i + c]);
        }
    double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-300});
    std::vector<std::pair<uint64_t, int32_t>> mk(nv);
    parallel_for(nv, 1 << 16, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i) {
            uint64_t q[3];
            for (int c = 0; c < 3; ++c) {
                double r = (xyz[3 * i + c] - lo[c]) / ext;
                q[c] = (uint64_t)std::min(2097151.0, std::max(0.0, std::floor(r * 2097151.0)));
            }
            mk[i] = {spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2), (int32_t)i};
        }
    });
    // (key, vertex) pairs are distinct: a total order
    parallel_sort(mk, [](const std::pair<uint64_t, int32_t>& a, const std::pair<uint64_t, int32_t>& b) {
        return a < b;
    });

    // ---- tiles: breadth-first region growing over the caller's one-ring
    // adjacency, seeded at the first unassigned vertex in Morton order; each
    // tile is connected and holds at most patch_size vertices.  The internal
    // vertex order is tile-major, breadth-first inside a tile.
    const int P = patch_size;
    const int parts = host_threads();
    std::vector<int32_t> order_v;
    order_v.reserve(nv);
    T.tile_ptr.clear();
    {
        // a vertex's neighbours in face order (two per incident face); each
        // worker fills the lists of its own range of vertices
        std::vector<int32_t> deg(nv + 1, 0);
        parallel_parts(nv, parts, [&](int64_t v0, int64_t v1, int) {
            for (int64_t i = 0; i < 3 * nf; ++i) {
                const int32_t a = tri_in[i];
                if (a >= v0 && a < v1) deg[a + 1] += 2;
            }
        });
        for (int64_t i = 0; i < nv; ++i) deg[i + 1] += deg[i];
        std::vector<int32_t> adj(deg[nv]);
        parallel_parts(nv, parts, [&](int64_t v0, int64_t v1, int) {
            std::vector<int32_t> pos(deg.begin() + v0, deg.begin() + v1);
            for (int64_t f = 0; f < nf; ++f)
                for (int k = 0; k < 3; ++k) {
                    const int32_t a = tri_in[3 * f + k], b = tri_in[3 * f + (k + 1) % 3];
                    if (a >= v0 && a < v1) adj[pos[a - v0]++] = b;
                    if (b >= v0 && b < v1) adj[pos[b - v0]++] = a;
                }
        });
        std::vector<int32_t> assigned(nv, -1);
        std::vector<int32_t> queue;
        queue.reserve(P);
        int32_t tile = 0;
        for (int64_t r = 0; r < nv; ++r) {
            int32_t seed = mk[r].second;
            if (assigned[seed] >= 0) continue;
            T.tile_ptr.push_back((int32_t)order_v.size());
            queue.clear();
            queue.push_back(seed);
            assigned[seed] = tile;
            for (size_t qi = 0; qi < queue.size() && (int)queue.size() < P; ++qi) {
                int32_t x = queue[qi];
                for (int32_t k = deg[x]; k < deg[x + 1] && (int)queue.size() < P; ++k) {
                    int32_t y = adj[k];
                    if (assigned[y] < 0) {
                        assigned[y] = tile;
                        queue.push_back(y);
                    }
                }
            }
            order_v.insert(order_v.end(), queue.begin(), queue.end());
            ++tile;
        }
        T.tile_ptr.push_back((int32_t)order_v.size());
    }
    T.perm_v.resize(nv);
    T.iperm_v.resize(nv);
    T.px.resize(nv);
    T.py.resize(nv);
    T.pz.resize(nv);
    parallel_for(nv, 1 << 16, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i) {
            int32_t u = order_v[i];
            T.perm_v[i] = u;
            T.iperm_v[u] = (int32_t)i;
            T.px[i] = xyz[3 * u];
            T.py[i] = xyz[3 * u + 1];
            T.pz[i] = xyz[3 * u + 2];
        }
    });
    mk.clear();
    mk.shrink_to_fit();

    // ---- faces sorted (stably) by smallest internal vertex
    {
        std::vector<int32_t> key(nf), fptr;
        parallel_for(nf, 1 << 16, [&](int64_t b, int64_t e) {
            for (int64_t f = b; f < e; ++f)
                key[f] = std::min({T.iperm_v[tri_in[3 * f]], T.iperm_v[tri_in[3 * f + 1]],
                                   T.iperm_v[tri_in[3 * f + 2]]});
        });
        group_by_key(key, nv, fptr, T.perm_f);
    }
    T.tri.resize(3 * nf);
    parallel_for(nf, 1 << 16, [&](int64_t b, int64_t e) {
        for (int64_t f = b; f < e; ++f) {
            int32_t u = T.perm_f[f];
            for (int k = 0; k < 3; ++k) T.tri[3 * f + k] = T.iperm_v[tri_in[3 * u + k]];
        }
    });

    // ---- halfedges bucketed by smaller internal endpoint
    const int64_t nh = 3 * nf;
    auto hend = [&](int64_t h) { return T.tri[(h / 3) * 3 + (h % 3 + 1) % 3]; };
    std::vector<int32_t> hptr, hb;
    {
        std::vector<int32_t> key(nh);
        parallel_for(nh, 1 << 16, [&](int64_t b, int64_t e) {
            for (int64_t h = b; h < e; ++h) key[h] = std::min(T.tri[h], hend(h));
        });
        group_by_key(key, nv, hptr, hb);
    }
    auto hother = [&](int32_t h) { return std::max(T.tri[h], hend(h)); };
    // within a bucket: order by larger endpoint, then halfedge id
    parallel_for(nv, 1 << 14, [&](int64_t vb, int64_t ve) {
        for (int64_t v = vb; v < ve; ++v)
            std::sort(hb.begin() + hptr[v], hb.begin() + hptr[v + 1], [&](int32_t x, int32_t y) {
                int32_t ox = hother(x), oy = hother(y);
                return ox != oy ? ox < oy : x < y;
            });
    });
    // unique edges: a group of equal (smaller, larger) endpoints never
    // leaves its bucket, so each worker numbers the groups of a range of
    // buckets; a first pass counts them (and finds the first invalid edge),
    // the second writes them at the worker's offset
    T.fslot.assign(nh, 0);
    T.fsign.assign(nf, 0);
    int64_t ne = 0, nbnd = 0;
    {
        std::vector<int64_t> pne(parts + 1, 0), pbnd(parts, 0);
        std::vector<int> perr(parts, 0);   // 1 non-manifold, 2 inconsistent orientation
        std::vector<uint8_t> tailbit(nh, 0);
        auto groups = [&](int64_t v0, int64_t v1, int p, bool write) {
            int64_t n = 0, nb = 0;
            for (int64_t i = hptr[v0]; i < hptr[v1];) {
                int32_t h0 = hb[i];
                int32_t a0 = T.tri[h0], b0 = hend(h0);
                int32_t lo_v = std::min(a0, b0), hi_v = std::max(a0, b0);
                int64_t j = i + 1;
                while (j < hptr[v1]) {
                    int32_t h1 = hb[j];
                    int32_t a1 = T.tri[h1], b1 = hend(h1);
                    if (std::min(a1, b1) != lo_v || std::max(a1, b1) != hi_v) break;
                    ++j;
                }
                const int64_t m = j - i;
                if (!write) {
                    if (m > 2) {
                        perr[p] = 1;
                        return;
                    }
                    if (m == 2 && a0 == T.tri[hb[i + 1]]) {
                        perr[p] = 2;
                        return;
                    }
                    if (m == 1) ++nb;
                } else {
                    // orientation halfedge: from the smaller to the larger caller id
                    const int32_t tail = T.perm_v[lo_v] < T.perm_v[hi_v] ? lo_v : hi_v;
                    const int32_t head = tail == lo_v ? hi_v : lo_v;
                    const int64_t e = pne[p] + n;
                    T.ev[2 * e] = tail;
                    T.ev[2 * e + 1] = head;
                    for (int64_t s = 0; s < 2; ++s) {
                        if (s < m) {
                            const int32_t h = hb[i + s];
                            T.ef[2 * e + s] = h / 3;
                            T.fslot[h] = ((uint32_t)e << 2) | ((m == 1 ? 1u : 0u) << 1) | (uint32_t)s;
                            tailbit[h] = T.tri[h] == tail;
                        } else {
                            T.ef[2 * e + s] = -1;
                        }
                    }
                }
                ++n;
                i = j;
            }
            if (!write) {
                pne[p + 1] = n;
                pbnd[p] = nb;
            }
        };
        parallel_parts(nv, parts, [&](int64_t v0, int64_t v1, int p) { groups(v0, v1, p, false); });
        for (int p = 0; p < parts; ++p) {
            if (perr[p] == 1) bad("non-manifold edge (more than two incident faces)");
            if (perr[p] == 2) bad("inconsistently oriented faces share an edge");
        }
        for (int p = 0; p < parts; ++p) {
            pne[p + 1] += pne[p];
            nbnd += pbnd[p];
        }
        ne = pne[parts];
        if (ne >= (1ll << 30)) throw Error{HG_E_INVALID_ARG, "too many edges"};
        T.ev.assign(2 * ne, 0);
        T.ef.assign(2 * ne, 0);
        parallel_parts(nv, parts, [&](int64_t v0, int64_t v1, int p) { groups(v0, v1, p, true); });
        parallel_for(nf, 1 << 16, [&](int64_t b, int64_t e) {
            for (int64_t f = b; f < e; ++f)
                T.fsign[f] = (uint8_t)(tailbit[3 * f] | (tailbit[3 * f + 1] << 1) | (tailbit[3 * f + 2] << 2));
        });
    }
    T.ne = ne;
    T.nbnd = nbnd;
    hb.clear();
    hb.shrink_to_fit();
    hptr.clear();
    hptr.shrink_to_fit();

    // ---- internal edge order: by owning face (the side-0 face, which has the
    //      smaller internal id), then slot, so consecutive faces touch mostly
    //      consecutive edges
    {
        std::vector<int32_t> nid(ne, -1);
        std::vector<int64_t> pcnt(parts + 1, 0);
        parallel_parts(nh, parts, [&](int64_t b, int64_t e, int p) {
            int64_t c = 0;
            for (int64_t h = b; h < e; ++h) c += (T.fslot[h] & 1u) == 0u;
            pcnt[p + 1] = c;
        });
        for (int p = 0; p < parts; ++p) pcnt[p + 1] += pcnt[p];
        parallel_parts(nh, parts, [&](int64_t b, int64_t e, int p) {
            int32_t next = (int32_t)pcnt[p];
            for (int64_t h = b; h < e; ++h) {
                uint32_t sl = T.fslot[h];
                if ((sl & 1u) == 0u) nid[sl >> 2] = next++;
            }
        });
        std::vector<int32_t> ev2(2 * ne), ef2(2 * ne);
        parallel_for(ne, 1 << 16, [&](int64_t b, int64_t eend) {
            for (int64_t e = b; e < eend; ++e) {
                int32_t n = nid[e];
                ev2[2 * n] = T.ev[2 * e];
                ev2[2 * n + 1] = T.ev[2 * e + 1];
                ef2[2 * n] = T.ef[2 * e];
                ef2[2 * n + 1] = T.ef[2 * e + 1];
            }
        });
        T.ev.swap(ev2);
        T.ef.swap(ef2);
        parallel_for(nh, 1 << 16, [&](int64_t b, int64_t e) {
            for (int64_t h = b; h < e; ++h) {
                uint32_t sl = T.fslot[h];
                T.fslot[h] = ((uint32_t)nid[sl >> 2] << 2) | (sl & 3u);
            }
        });
    }

    // ---- slot twins
    {
        T.h01.assign(2 * ne, -1);
        parallel_for(nh, 1 << 16, [&](int64_t b, int64_t e) {
            for (int64_t h = b; h < e; ++h) {
                uint32_t sl = T.fslot[h];
                T.h01[2 * (sl >> 2) + (sl & 1u)] = (int32_t)h;
            }
        });
        T.twin.assign(nh, -1);
        parallel_for(ne, 1 << 16, [&](int64_t b, int64_t eend) {
            for (int64_t e = b; e < eend; ++e)
                if (T.h01[2 * e + 1] >= 0) {
                    T.twin[T.h01[2 * e]] = T.h01[2 * e + 1];
                    T.twin[T.h01[2 * e + 1]] = T.h01[2 * e];
                }
        });
    }

    // ---- canonical edge numbering: sort by (min caller id, max caller id)
    {
        auto umin = [&](int64_t e) { return std::min(T.perm_v[T.ev[2 * e]], T.perm_v[T.ev[2 * e + 1]]); };
        auto umax = [&](int64_t e) { return std::max(T.perm_v[T.ev[2 * e]], T.perm_v[T.ev[2 * e + 1]]); };
        std::vector<int32_t> key(ne), c2, order;
        parallel_for(ne, 1 << 16, [&](int64_t b, int64_t e) {
            for (int64_t x = b; x < e; ++x) key[x] = umin(x);
        });
        group_by_key(key, nv, c2, order);
        parallel_for(nv, 1 << 14, [&](int64_t vb, int64_t ve) {
            for (int64_t v = vb; v < ve; ++v)
                std::sort(order.begin() + c2[v], order.begin() + c2[v + 1],
                          [&](int32_t x, int32_t y) { return umax(x) < umax(y); });
        });
        T.perm_e.assign(ne, 0);
        parallel_for(ne, 1 << 16, [&](int64_t b, int64_t e) {
            for (int64_t r = b; r < e; ++r) T.perm_e[order[r]] = (int32_t)r;
        });
    }

    // ---- CSR adjacency in internal order, neighbours sorted by internal id
    T.row_ptr.assign(nv + 1, 0);
    parallel_parts(nv, parts, [&](int64_t v0, int64_t v1, int) {
        for (int64_t i = 0; i < 2 * ne; ++i) {
            const int32_t a = T.ev[i];
            if (a >= v0 && a < v1) T.row_ptr[a + 1]++;
        }
    });
    for (int64_t i = 0; i < nv; ++i) T.row_ptr[i + 1] += T.row_ptr[i];
    T.col.assign(2 * ne, 0);
    T.csr_edge.assign(2 * ne, 0);
    parallel_parts(nv, parts, [&](int64_t v0, int64_t v1, int) {
        std::vector<int32_t> pos(T.row_ptr.begin() + v0, T.row_ptr.begin() + v1);
        for (int64_t e = 0; e < ne; ++e) {
            const int32_t a = T.ev[2 * e], b = T.ev[2 * e + 1];
            if (a >= v0 && a < v1) {
                T.col[pos[a - v0]] = b;
                T.csr_edge[pos[a - v0]++] = (int32_t)e;
            }
            if (b >= v0 && b < v1) {
                T.col[pos[b - v0]] = a;
                T.csr_edge[pos[b - v0]++] = (int32_t)e;
            }
        }
    });
    {
        std::vector<int> pmax(parts, 0);
        parallel_parts(nv, parts, [&](int64_t vb, int64_t ve, int p) {
            std::vector<std::pair<int32_t, int32_t>> tmp;
            int maxdeg = 0;
            for (int64_t v = vb; v < ve; ++v) {
                int32_t b = T.row_ptr[v], e = T.row_ptr[v + 1];
                maxdeg = std::max(maxdeg, e - b);
                tmp.clear();
                for (int32_t k = b; k < e; ++k) tmp.push_back({T.col[k], T.csr_edge[k]});
                std::sort(tmp.begin(), tmp.end());
                for (int32_t k = b; k < e; ++k) {
                    T.col[k] = tmp[k - b].first;
                    T.csr_edge[k] = tmp[k - b].second;
                }
            }
            pmax[p] = maxdeg;
        });
        T.max_valence = *std::max_element(pmax.begin(), pmax.end());
    }

    // ---- LDS tiles: halos and ELL local slots of the tiles built above.
    //      Per tile in parallel: its halo and ELL width; then the offsets (and
    //      the first invalid tile, in tile order); then the tables.
    T.patch_size = P;
    const int64_t np = (int64_t)T.tile_ptr.size() - 1;
    T.halo_ptr.assign(np + 1, 0);
    T.ell_ptr.assign(np + 1, 0);
    T.ell_width.assign(np, 0);
    T.max_halo = 0;
    T.max_ell_width = 0;
    {
        std::vector<std::vector<int32_t>> halos(np);
        std::vector<int32_t> width(np, 0);
        parallel_for(np, 16, [&](int64_t pb, int64_t pe) {
            for (int64_t p = pb; p < pe; ++p) {
                const int64_t v0 = T.tile_ptr[p], v1 = T.tile_ptr[p + 1];
                auto& halo = halos[p];
                int w = 0;
                for (int64_t v = v0; v < v1; ++v) {
                    w = std::max(w, T.row_ptr[v + 1] - T.row_ptr[v]);
                    for (int32_t k = T.row_ptr[v]; k < T.row_ptr[v + 1]; ++k) {
                        int32_t u = T.col[k];
                        if (u < v0 || u >= v1) halo.push_back(u);
                    }
                }
                std::sort(halo.begin(), halo.end());
                halo.erase(std::unique(halo.begin(), halo.end()), halo.end());
                width[p] = w;
            }
        });
        int64_t base = 0;
        for (int64_t p = 0; p < np; ++p) {
            if ((int64_t)P + (int64_t)halos[p].size() >= 65535)
                throw Error{HG_E_BAD_MESH, "tile halo too large for 16-bit local slots"};
            T.halo_ptr[p + 1] = T.halo_ptr[p] + (int32_t)halos[p].size();
            T.max_halo = std::max<int>(T.max_halo, (int)halos[p].size());
            T.ell_width[p] = (uint8_t)std::min(width[p], 255);
            if (width[p] > 255) throw Error{HG_E_BAD_MESH, "vertex valence above 255"};
            T.max_ell_width = std::max(T.max_ell_width, width[p]);
            T.ell_ptr[p] = (int32_t)base;
            base += (int64_t)width[p] * P;
            if (base >= (1ll << 31)) throw Error{HG_E_INVALID_ARG, "tile table too large"};
        }
        T.ell_ptr[np] = (int32_t)base;
        T.halo_idx.assign(T.halo_ptr[np], 0);
        T.lnb.assign(base, (uint16_t)0xFFFF);
        parallel_for(np, 16, [&](int64_t pb, int64_t pe) {
            for (int64_t p = pb; p < pe; ++p) {
                const int64_t v0 = T.tile_ptr[p], v1 = T.tile_ptr[p + 1];
                const auto& halo = halos[p];
                std::copy(halo.begin(), halo.end(), T.halo_idx.begin() + T.halo_ptr[p]);
                const int64_t b = T.ell_ptr[p];
                for (int64_t v = v0; v < v1; ++v) {
                    int i = (int)(v - v0);
                    int s = 0;
                    for (int32_t k = T.row_ptr[v]; k < T.row_ptr[v + 1]; ++k, ++s) {
                        int32_t u = T.col[k];
                        uint16_t l;
                        if (u >= v0 && u < v1) {
                            l = (uint16_t)(u - v0);
                        } else {
                            l = (uint16_t)(P + (std::lower_bound(halo.begin(), halo.end(), u) - halo.begin()));
                        }
                        T.lnb[b + (int64_t)s * P + i] = l;
                    }
                }
            }
        });
    }

    // ---- tile adjacency: a tile's halo lies in its neighbour tiles
    std::vector<int32_t> tile_of(nv);
    parallel_for(np, 16, [&](int64_t pb, int64_t pe) {
        for (int64_t p = pb; p < pe; ++p)
            for (int32_t v = T.tile_ptr[p]; v < T.tile_ptr[p + 1]; ++v) tile_of[v] = (int32_t)p;
    });
    std::vector<std::vector<int32_t>> adj(np);
    for (int64_t p = 0; p < np; ++p)
        for (int32_t h = T.halo_ptr[p]; h < T.halo_ptr[p + 1]; ++h) {
            const int32_t q = tile_of[T.halo_idx[h]];
            adj[p].push_back(q);
            adj[q].push_back((int32_t)p);
        }
    parallel_for(np, 64, [&](int64_t pb, int64_t pe) {
        for (int64_t p = pb; p < pe; ++p) {
            auto& a = adj[p];
            std::sort(a.begin(), a.end());
            a.erase(std::unique(a.begin(), a.end()), a.end());
        }
    });

    // ---- connected components (several meshes may be packed into one):
    //      tiles are connected, so the components are those of the tile
    //      graph; numbered in the order of their smallest caller vertex id
    {
        std::vector<int32_t> tc(np, -1), stack;
        int nc = 0;
        for (int64_t p0 = 0; p0 < np; ++p0) {
            if (tc[p0] >= 0) continue;
            tc[p0] = nc;
            stack.assign(1, (int32_t)p0);
            while (!stack.empty()) {
                const int32_t p = stack.back();
                stack.pop_back();
                for (int32_t q : adj[p])
                    if (tc[q] < 0) {
                        tc[q] = nc;
                        stack.push_back(q);
                    }
            }
            ++nc;
        }
        std::vector<int32_t> tile_lo(np);
        parallel_for(np, 16, [&](int64_t pb, int64_t pe) {
            for (int64_t p = pb; p < pe; ++p) {
                int32_t lo = 0x7fffffff;
                for (int32_t v = T.tile_ptr[p]; v < T.tile_ptr[p + 1]; ++v) lo = std::min(lo, T.perm_v[v]);
                tile_lo[p] = lo;
            }
        });
        std::vector<int32_t> first_caller(nc, 0x7fffffff);
        for (int64_t p = 0; p < np; ++p) first_caller[tc[p]] = std::min(first_caller[tc[p]], tile_lo[p]);
        std::vector<int32_t> ord(nc), rank(nc);
        for (int c = 0; c < nc; ++c) ord[c] = c;
        std::sort(ord.begin(), ord.end(), [&](int a, int b) { return first_caller[a] < first_caller[b]; });
        for (int c = 0; c < nc; ++c) rank[ord[c]] = c;
        T.n_comp = nc;
        T.tile_comp.assign(np, 0);
        for (int64_t p = 0; p < np; ++p) T.tile_comp[p] = rank[tc[p]];
        T.comp.assign(nv, -1);
        parallel_for(nv, 1 << 16, [&](int64_t b, int64_t e) {
            for (int64_t v = b; v < e; ++v) T.comp[v] = T.tile_comp[tile_of[v]];
        });
        // mean edge length per component, summed in edge order
        std::vector<double> len(nc, 0.0);
        std::vector<int64_t> cnt(nc, 0);
        for (int64_t e = 0; e < ne; ++e) {
            int32_t a = T.ev[2 * e], b = T.ev[2 * e + 1];
            double dx = T.px[a] - T.px[b], dy = T.py[a] - T.py[b], dz = T.pz[a] - T.pz[b];
            len[T.comp[a]] += std::sqrt(dx * dx + dy * dy + dz * dz);
            cnt[T.comp[a]]++;
        }
        T.comp_hbar.assign(nc, 0.0);
        for (int c = 0; c < nc; ++c) T.comp_hbar[c] = cnt[c] ? len[c] / (double)cnt[c] : 0.0;
    }

    // ---- colouring of the tiles: tiles of one colour never read each other
    {
        colour_tiles(adj, T.color_ptr, T.tile_order, slots);
        T.tile_adj_ptr.assign(np + 1, 0);
        for (int64_t p = 0; p < np; ++p) T.tile_adj_ptr[p + 1] = T.tile_adj_ptr[p] + (int32_t)adj[p].size();
        T.tile_adj.clear();
        T.tile_adj.reserve(T.tile_adj_ptr[np]);
        for (const auto& a : adj) T.tile_adj.insert(T.tile_adj.end(), a.begin(), a.end());
    }
}

void colour_tiles(const std::vector<std::vector<int32_t>>& adj, std::vector<int32_t>& color_ptr,
                  std::vector<int32_t>& order, int slots) {
    const int64_t n = (int64_t)adj.size();
    std::vector<int32_t> color(n, -1);
    // per node: the set of its neighbours' colours (a bit mask while the
    // colours fit 64 bits, a list beyond) and its saturation (their count)
    std::vector<uint64_t> seen(n, 0);
    std::vector<std::vector<int32_t>> seen_hi(n);
    std::vector<int32_t> sat(n, 0);
    auto has = [&](int64_t v, int c) {
        if (c < 64) return ((seen[v] >> c) & 1u) != 0;
        return std::find(seen_hi[v].begin(), seen_hi[v].end(), c) != seen_hi[v].end();
    };
    // pick: largest saturation, then largest degree, then smallest index;
    // a max-heap with lazy deletion of stale entries
    struct Key {
        int32_t sat, deg;
        int64_t v;
        bool operator<(const Key& o) const {
            if (sat != o.sat) return sat < o.sat;
            if (deg != o.deg) return deg < o.deg;
            return v > o.v;
        }
    };
    std::vector<Key> heap;
    heap.reserve(n);
    for (int64_t v = 0; v < n; ++v) heap.push_back({0, (int32_t)adj[v].size(), v});
    std::make_heap(heap.begin(), heap.end());
    int ncol = 0;
    while (!heap.empty()) {
        std::pop_heap(heap.begin(), heap.end());
        const Key k = heap.back();
        heap.pop_back();
        const int64_t v = k.v;
        if (color[v] >= 0 || k.sat != sat[v]) continue;   // stale
        int c = 0;
        while (has(v, c)) ++c;
        color[v] = c;
        ncol = std::max(ncol, c + 1);
        for (int32_t u : adj[v]) {
            if (color[u] >= 0 || has(u, c)) continue;
            if (c < 64)
                seen[u] |= (uint64_t)1 << c;
            else
                seen_hi[u].push_back(c);
            heap.push_back({++sat[u], (int32_t)adj[u].size(), u});
            std::push_heap(heap.begin(), heap.end());
        }
    }
    // waves: trim each colour's overflow past a multiple of slots (up to a
    // half of slots) into colours with room, nodes in index order
    if (slots > 0 && ncol > 1) {
        std::vector<int64_t> size(ncol, 0);
        for (int64_t v = 0; v < n; ++v) size[color[v]]++;
        std::vector<char> nbc(ncol);
        for (int c = 0; c < ncol; ++c) {
            const int64_t over = size[c] % slots;
            if (over == 0 || over > slots / 2 || size[c] <= slots) continue;
            for (int64_t v = 0; v < n && size[c] % slots != 0; ++v) {
                if (color[v] != c) continue;
                std::fill(nbc.begin(), nbc.end(), 0);
                for (int32_t u : adj[v]) nbc[color[u]] = 1;
                int best = -1;
                int64_t room = 0;
                for (int j = 0; j < ncol; ++j) {
                    if (j == c || nbc[j] || size[j] % slots == 0) continue;
                    const int64_t r = slots - size[j] % slots;
                    if (r > room) {
                        room = r;
                        best = j;
                    }
                }
                if (best < 0) continue;
                color[v] = best;
                size[c]--;
                size[best]++;
            }
        }
    }
    color_ptr.assign(ncol + 1, 0);
    for (int64_t v = 0; v < n; ++v) color_ptr[color[v] + 1]++;
    for (int c = 0; c < ncol; ++c) color_ptr[c + 1] += color_ptr[c];
    order.assign(n, 0);
    std::vector<int32_t> pos(color_ptr.begin(), color_ptr.end() - 1);
    for (int64_t v = 0; v < n; ++v) order[pos[color[v]]++] = (int32_t)v;
}

}  // namespace hg
