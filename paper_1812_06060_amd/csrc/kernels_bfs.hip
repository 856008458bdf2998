// Breadth-first vertex sets D_i (Eq. 6) and the pairing of every vertex with
// a neighbour one set closer to the sources (Sec. 3.3; Sec. 5.2 puts all
// sources in D_0).  Two schedules give the same levels: on meshes with
// diffusion tiles, min-plus relaxation over the tiles (below); otherwise
// level-synchronous frontier expansion, one launch per level, frontier
// membership claimed with atomicCAS on the level array (the levels are
// unique, so the result does not depend on timing).  The pairing is then
// chosen per vertex as the neighbour of level - 1 with the smallest caller
// vertex id, which is deterministic.
#include "hgeo_internal.h"

namespace hg {

constexpr int kBlockB = 256;

__global__ void k_fill_i32(int n, int32_t* a, int32_t val) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = val;
}

// counters[0..2]: frontier sizes (ring of three), counters[3]: depth
__global__ void k_bfs_sources(int nsrc, const int32_t* src, int32_t* level, int32_t* frontier, int32_t* counters) {
    if (blockIdx.x != 0) return;
    if (threadIdx.x == 0) {
        int n = 0;
        for (int i = 0; i < nsrc; ++i) {
            int s = src[i];
            if (level[s] < 0) {
                level[s] = 0;
                frontier[n++] = s;
            }
        }
        counters[0] = n;
        counters[1] = 0;
        counters[2] = 0;
        counters[3] = 0;
    }
}

// One level's expansion: the vertices of frontier L claim their unvisited
// neighbours for level L + 1 (atomicCAS on the level array) and append them
// to the next frontier, one atomic per wavefront.
__global__ void k_bfs_expand(int L, int nv, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                             int32_t* level, const int32_t* fin, int32_t* fout, int32_t* counters) {
    const int cin = L % 3, cout = (L + 1) % 3, czero = (L + 2) % 3;
    const int n = min(counters[cin], nv);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        counters[czero] = 0;
        if (n > 0) counters[3] = L;   // deepest non-empty level so far
    }
    const int lane = threadIdx.x & 63;
    const int stride = gridDim.x * blockDim.x;
    constexpr int kCap = 16;
    // the loop bound is uniform across a wavefront, so every lane reaches
    // the shuffles below
    for (int base = blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < n; base += stride) {
        int i = base + lane;
        int claimed[kCap];
        int c = 0;
        const int v = i < n ? fin[i] : -1;
        if (v >= 0 && v < nv) {
            for (int k = row_ptr[v]; k < row_ptr[v + 1]; ++k) {
                int u = col[k];
                if (level[u] < 0 && atomicCAS(&level[u], -1, L + 1) == -1) {
                    if (c < kCap) {
                        claimed[c++] = u;
                    } else {
                        int pos = atomicAdd(&counters[cout], 1);
                        fout[pos] = u;
                    }
                }
            }
        }
        // wavefront prefix sum of the claim counts, one atomic per wavefront
        int incl = c;
        for (int o = 1; o < 64; o <<= 1) {
            int t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        int total = __shfl(incl, 63, 64);
        int wbase = 0;
        if (lane == 63 && total > 0) wbase = atomicAdd(&counters[cout], total);
        wbase = __shfl(wbase, 63, 64);
        int off = wbase + incl - c;
        for (int q = 0; q < c; ++q) fout[off + q] = claimed[q];
    }
}

// Each reached vertex's partner in the previous set (the neighbour of smallest
// caller id) and the edge to it, -1 for sources and unreached vertices.
__global__ void k_bfs_parent(int nv, const int32_t* row_ptr, const int32_t* col, const int32_t* csr_edge,
                             const int32_t* level, const int32_t* perm_v, int32_t* parent, int32_t* pedge) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nv) return;
    int lj = level[j];
    int best = -1, bslot = -1, bid = 0x7fffffff;
    if (lj > 0) {
        for (int k = row_ptr[j]; k < row_ptr[j + 1]; ++k) {
            int u = col[k];
            if (level[u] == lj - 1) {
                int id = perm_v[u];
                if (id < bid) {
                    bid = id;
                    best = u;
                    bslot = k;
                }
            }
        }
    }
    parent[j] = best;
    pedge[j] = bslot >= 0 ? csr_edge[bslot] : -1;
}

int run_bfs_into(Mesh& m, const BfsBuffers& b, const std::vector<int32_t>& src, hipStream_t s) {
    const int nv = (int)m.nv;
    HG_CHECK_HIP(hipMemcpyAsync(b.src, src.data(), src.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(nv, kBlockB)), dim3(kBlockB), 0, s, nv, b.level, -1);
    hipLaunchKernelGGL(k_bfs_sources, dim3(1), dim3(64), 0, s, (int)src.size(), b.src, b.level, b.frontier_a,
                       b.counters);
    HG_CHECK_HIP(hipGetLastError());
    int32_t hc[4];
    // The grid follows the frontier size last read back (twice it, in
    // threads): a launch of far more workgroups than frontier vertices costs
    // more than the expansion itself.  A frontier that has grown since is
    // still covered, by the kernel's grid-stride loop.
    const int max_grid = std::max(1, std::min(grid_for(nv, kBlockB), 2048));
    auto grid_for_frontier = [&](int64_t n) {
        const int64_t g = (2 * n + kBlockB - 1) / kBlockB;
        return (int)std::max<int64_t>(std::min(8, max_grid), std::min<int64_t>(max_grid, g));
    };
    int grid = grid_for_frontier((int64_t)src.size() * 64);
    for (int L = 0;; ++L) {
        int32_t* fin = (L % 2 == 0) ? b.frontier_a : b.frontier_b;
        int32_t* fout = (L % 2 == 0) ? b.frontier_b : b.frontier_a;
        hipLaunchKernelGGL(k_bfs_expand, dim3(grid), dim3(kBlockB), 0, s, L, nv, m.row_ptr.p, m.col.p, b.level,
                           fin, fout, b.counters);
        HG_CHECK_HIP(hipGetLastError());
        if ((L & 31) == 31) {
            HG_CHECK_HIP(hipMemcpyAsync(hc, b.counters, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HG_CHECK_HIP(hipStreamSynchronize(s));
            if (hc[(L + 1) % 3] == 0) break;
            grid = grid_for_frontier(hc[(L + 1) % 3]);
        }
        if (L > nv + 1) break;
    }
    hipLaunchKernelGGL(k_bfs_parent, dim3(grid_for(nv, kBlockB)), dim3(kBlockB), 0, s, nv, m.row_ptr.p, m.col.p,
                       m.csr_edge.p, b.level, m.perm_v.p, b.parent, b.pedge);
    HG_CHECK_HIP(hipGetLastError());
    HG_CHECK_HIP(hipMemcpyAsync(hc, b.counters, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HG_CHECK_HIP(hipStreamSynchronize(s));
    return hc[3];   // deepest level whose frontier was non-empty
}

// ---------------------------------------------------------------- tiled
// The same levels as the shortest hop counts from the sources (D_i = the
// vertices at hop distance i, Eq. 6), found by min-plus relaxation
// level_j = min(level_j, level_k + 1) over the diffusion tiles: per colour
// one launch, each tile relaxing its vertices in LDS until nothing changes
// (its halo held), passes until no tile changes over a whole pass.  The
// fixed point is unique, so the levels equal the level-synchronous search's
// exactly; about depth / (rings crossed per pass) passes instead of depth
// dependent launches.  The pairing is chosen afterwards as before.
// A tile works in pass k only if it or a neighbour tile changed in pass
// k - 1 or earlier in pass k (mark >= k - 1): elsewhere nothing can move,
// so the other tiles cost one read of their mark (k_bfs_tiles).
constexpr int kTileB = 1024;         // vertices per diffusion tile
constexpr int32_t kFar = 0x3fffffff;   // not reached (yet)

// One tile's relaxation (the whole workgroup; lv: its LDS levels).
template <int MAXW>
__device__ __forceinline__ void bfs_tile_body(int p, const int32_t* __restrict__ tile_ptr,
                                              const int32_t* __restrict__ halo_ptr,
                                              const int32_t* __restrict__ halo_idx,
                                              const int32_t* __restrict__ ell_ptr,
                                              const uint8_t* __restrict__ ell_width,
                                              const uint16_t* __restrict__ lnb, const int32_t* __restrict__ adj_ptr,
                                              const int32_t* __restrict__ adj, int32_t* level, int32_t* mark,
                                              int pass, int32_t* changes, int32_t* lv) {
    const int v0 = tile_ptr[p], np = tile_ptr[p + 1] - v0;
    const int h0 = halo_ptr[p], nh = halo_ptr[p + 1] - h0;
    const int W = ell_width[p], eb = ell_ptr[p];
    const int tid = threadIdx.x;
    const bool in = tid < np;
    int own = in ? level[v0 + tid] : kFar;
    uint16_t l[MAXW];
#pragma unroll
    for (int k = 0; k < MAXW; ++k) {
        const bool ok = in && k < W;
        const uint16_t li = ok ? lnb[eb + k * kTileB + tid] : (uint16_t)0xFFFF;
        l[k] = li != 0xFFFF ? li : (uint16_t)tid;   // padding reads the own slot: no effect
    }
    for (int j = tid; j < nh; j += kTileB) lv[kTileB + j] = level[halo_idx[h0 + j]];
    lv[tid] = own;
    __syncthreads();
    const int start = own;
    // in-place updates in any order reach the same least fixed point; it is
    // reached within as many rounds as the tile has vertices
    for (int round = 0; round <= kTileB; ++round) {
        int best = own;
#pragma unroll
        for (int k = 0; k < MAXW; ++k) best = min(best, lv[l[k]] + 1);
        const int ch = best < own;
        if (ch) {
            own = best;
            lv[tid] = best;
        }
        if (!__syncthreads_or(ch)) break;
    }
    const int moved = in && own != start;
    if (moved) level[v0 + tid] = own;
    if (__syncthreads_or(moved)) {
        // the tile and its neighbours work in this pass (later colours)
        // and the next (earlier colours); every writer writes this pass
        const int a0 = adj_ptr[p], na = adj_ptr[p + 1] - a0;
        for (int k = tid; k < na; k += kTileB) mark[adj[a0 + k]] = pass;
        if (tid == 0) {
            mark[p] = pass;
            atomicAdd(changes, 1);
        }
    }
}

// One colour of one pass: workgroup b takes the colour's entries b, b + G,
// b + 2G, ... (G = gridDim.x; at most kTileB of them), keeps those whose
// tile is marked (mark >= pass - 1: it or a neighbour changed in the last
// pass or earlier in this one) and relaxes them one after the other.  Only
// the marked tiles cost more than one read.  The order within a workgroup
// does not matter: tiles of one colour never read what another writes.
template <int MAXW>
__global__ void __launch_bounds__(kTileB) k_bfs_tiles(const int32_t* __restrict__ tile_list, int nc,
                                                      const int32_t* __restrict__ tile_ptr,
                                                      const int32_t* __restrict__ halo_ptr,
                                                      const int32_t* __restrict__ halo_idx,
                                                      const int32_t* __restrict__ ell_ptr,
                                                      const uint8_t* __restrict__ ell_width,
                                                      const uint16_t* __restrict__ lnb,
                                                      const int32_t* __restrict__ adj_ptr,
                                                      const int32_t* __restrict__ adj, int32_t* level,
                                                      int32_t* mark, int pass, int32_t* changes, int lv_slots) {
    extern __shared__ int32_t lds[];   // levels (lv_slots: core, then halo), then the active list
    int32_t* lv = lds;
    int32_t* act = lds + lv_slots;
    __shared__ int n_act;
    const int tid = threadIdx.x;
    const int G = gridDim.x, b = blockIdx.x;
    if (tid == 0) n_act = 0;
    __syncthreads();
    const int i = b + tid * G;
    if (i < nc) {
        const int p = tile_list[i];
        if (mark[p] >= pass - 1) act[atomicAdd(&n_act, 1)] = p;
    }
    __syncthreads();
    const int na = n_act;
    for (int k = 0; k < na; ++k) {
        bfs_tile_body<MAXW>(act[k], tile_ptr, halo_ptr, halo_idx, ell_ptr, ell_width, lnb, adj_ptr, adj, level, mark,
                            pass, changes, lv);
        __syncthreads();   // the next tile rewrites lv
    }
}

// marks: -2 everywhere, -1 on the tiles holding a source (they work in pass 0)
__global__ void k_bfs_marks(int nt, int32_t* mark) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nt) mark[p] = -2;
}
__global__ void k_bfs_mark_sources(int nsrc, const int32_t* src, int nt, const int32_t* tile_ptr, int32_t* mark) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsrc) return;
    const int v = src[i];
    int lo = 0, hi = nt - 1;   // the tile p with tile_ptr[p] <= v < tile_ptr[p + 1]
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (tile_ptr[mid] <= v)
            lo = mid;
        else
            hi = mid - 1;
    }
    mark[lo] = -1;
}

__global__ void k_bfs_seed(int nv, int32_t* level, int32_t* counters) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nv) level[i] = kFar;
    if (i < 8) counters[i] = 0;
}
__global__ void k_bfs_seed_sources(int nsrc, const int32_t* src, int32_t* level) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nsrc) level[src[i]] = 0;
}
// unreached back to -1; each block's deepest level into blockmax, then the
// deepest of all into counters[3] (one block; no contended atomics)
__global__ void __launch_bounds__(kBlockB) k_bfs_tile_finish(int nv, int32_t* level, int32_t* blockmax) {
    __shared__ int32_t sh[kBlockB / 64];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int d = 0;
    if (i < nv) {
        const int v = level[i];
        if (v >= kFar)
            level[i] = -1;
        else
            d = v;
    }
    for (int o = 32; o > 0; o >>= 1) d = max(d, __shfl_down(d, o, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = d;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kBlockB / 64; ++k) d = max(d, sh[k]);
        blockmax[blockIdx.x] = d;
    }
}
__global__ void __launch_bounds__(1024) k_bfs_depth(int n, const int32_t* blockmax, int32_t* counters) {
    __shared__ int32_t sh[1024 / 64];
    int d = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) d = max(d, blockmax[i]);
    for (int o = 32; o > 0; o >>= 1) d = max(d, __shfl_down(d, o, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = d;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 1024 / 64; ++k) d = max(d, sh[k]);
        counters[3] = d;
    }
}

// The tiled search wins while the tiles are few: 16 against 35 ms at L10
// (10,487 tiles, depth 2,589), but 286 against 177 ms at L12 (164k tiles,
// depth 10-11k), where a pass's colour launches carry many more marked
// tiles; the level-synchronous search is used beyond 32,768 tiles.
constexpr int kMaxTilesTiledBfs = 32768;

static bool bfs_tiles_supported(const Mesh& m) {
    return m.patch_size == kTileB && m.n_patches > 0 && m.n_patches <= kMaxTilesTiledBfs && m.max_ell_width <= 16 &&
           m.tile_adj_ptr.n == (size_t)m.n_patches + 1 &&
           (size_t)(2 * kTileB + m.max_halo) * 4 <= 65536;
}

static int run_bfs_tiles(Mesh& m, const BfsBuffers& b, int32_t* mark, const std::vector<int32_t>& src,
                         hipStream_t s) {
    const int nv = (int)m.nv;
    HG_CHECK_HIP(hipMemcpyAsync(b.src, src.data(), src.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_bfs_seed, dim3(grid_for(std::max(nv, 8), kBlockB)), dim3(kBlockB), 0, s, nv, b.level,
                       b.counters);
    hipLaunchKernelGGL(k_bfs_seed_sources, dim3(grid_for((int64_t)src.size(), kBlockB)), dim3(kBlockB), 0, s,
                       (int)src.size(), b.src, b.level);
    const int nt = m.n_patches;
    hipLaunchKernelGGL(k_bfs_marks, dim3(grid_for(nt, kBlockB)), dim3(kBlockB), 0, s, nt, mark);
    hipLaunchKernelGGL(k_bfs_mark_sources, dim3(grid_for((int64_t)src.size(), kBlockB)), dim3(kBlockB), 0, s,
                       (int)src.size(), b.src, nt, m.tile_ptr.p, mark);
    HG_CHECK_HIP(hipGetLastError());
    const int lv_slots = kTileB + m.max_halo;
    const size_t lds = (size_t)(lv_slots + kTileB) * sizeof(int32_t);
    const int maxw = m.max_ell_width;
    const std::vector<int32_t>& cp = m.color_ptr_host;
    const int ncol = (int)cp.size() - 1;
    int dev = 0, cus = 0;
    HG_CHECK_HIP(hipGetDevice(&dev));
    HG_CHECK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int slots = std::max(1, 2 * cus);   // two 1024-thread workgroups per CU
    // a pass can move the front by as little as one ring, so depth + 1
    // passes always suffice; checks read the change count every few passes
    constexpr int kCheck = 4;
    int32_t hc[4];
    int32_t last = -1;
    for (int pass = 0;; ++pass) {
        for (int c = 0; c < ncol; ++c) {
            const int nc = cp[c + 1] - cp[c];
            if (nc == 0) continue;
            // one wave of workgroups, each scanning at most kTileB entries
            const int G = std::max(std::min(nc, slots), (nc + kTileB - 1) / kTileB);
#define HG_BFS_TILE_ARGS                                                                                      \
    dim3(G), dim3(kTileB), lds, s, m.tile_order.p + cp[c], nc, m.tile_ptr.p, m.halo_ptr.p, m.halo_idx.p,      \
        m.ell_ptr.p, m.ell_width.p, m.lnb.p, m.tile_adj_ptr.p, m.tile_adj.p, b.level, mark, pass, b.counters, \
        lv_slots
            if (maxw <= 6)
                hipLaunchKernelGGL(k_bfs_tiles<6>, HG_BFS_TILE_ARGS);
            else if (maxw <= 8)
                hipLaunchKernelGGL(k_bfs_tiles<8>, HG_BFS_TILE_ARGS);
            else
                hipLaunchKernelGGL(k_bfs_tiles<16>, HG_BFS_TILE_ARGS);
#undef HG_BFS_TILE_ARGS
        }
        HG_CHECK_HIP(hipGetLastError());
        if (pass % kCheck == kCheck - 1) {
            HG_CHECK_HIP(hipMemcpyAsync(hc, b.counters, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HG_CHECK_HIP(hipStreamSynchronize(s));
            if (hc[0] == last) break;   // no tile changed over the last kCheck passes
            last = hc[0];
        }
        if (pass > nv + kCheck) throw Error{HG_E_DEVICE, "tiled breadth-first search did not settle"};
    }
    // the frontier queue is free in this schedule: it holds the block maxima
    const int nb = grid_for(nv, kBlockB);
    hipLaunchKernelGGL(k_bfs_tile_finish, dim3(nb), dim3(kBlockB), 0, s, nv, b.level, b.frontier_a);
    hipLaunchKernelGGL(k_bfs_depth, dim3(1), dim3(1024), 0, s, nb, b.frontier_a, b.counters);
    hipLaunchKernelGGL(k_bfs_parent, dim3(grid_for(nv, kBlockB)), dim3(kBlockB), 0, s, nv, m.row_ptr.p, m.col.p,
                       m.csr_edge.p, b.level, m.perm_v.p, b.parent, b.pedge);
    HG_CHECK_HIP(hipGetLastError());
    HG_CHECK_HIP(hipMemcpyAsync(hc, b.counters, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HG_CHECK_HIP(hipStreamSynchronize(s));
    return hc[3];
}

int run_bfs(Mesh& m, Work& w, const std::vector<int32_t>& src, hipStream_t s) {
    const int nv = (int)m.nv;
    w.level.alloc(nv);
    w.parent.alloc(nv);
    w.pedge.alloc(nv);
    w.frontier_a.alloc(nv);
    w.frontier_b.alloc(nv);
    w.counters.alloc(8);
    w.src.alloc(src.size());
    BfsBuffers b{w.level.p, w.parent.p, w.pedge.p, w.frontier_a.p, w.frontier_b.p, w.counters.p, w.src.p};
    if (!bfs_tiles_supported(m)) return run_bfs_into(m, b, src, s);
    w.tile_mark.alloc((size_t)m.n_patches);
    return run_bfs_tiles(m, b, w.tile_mark.p, src, s);
}

}  // namespace hg
