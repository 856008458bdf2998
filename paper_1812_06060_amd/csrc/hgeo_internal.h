// Internal structures of the hgeo library (not part of the C ABI).
//
// Device layout of a resident mesh.  Vertices are renumbered internally tile
// by tile: tiles are connected patches of at most 1024 vertices grown
// breadth-first from seeds taken in 3D Morton order, so one-ring
// neighbourhoods sit close in memory and every tile is a compact surface
// patch; faces are sorted by their smallest internal vertex and edges by
// their internal endpoints.  The permutations back to the caller's order are
// kept on the device.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/hgeo.h"

namespace hg {

// Throwing helpers used inside the library; the C ABI converts to status.
struct Error {
    hg_status code;
    std::string msg;
};

#define HG_CHECK_HIP(expr)                                                                  \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess)                                                               \
            throw ::hg::Error{_e == hipErrorOutOfMemory ? HG_E_OOM : HG_E_DEVICE,           \
                              std::string(#expr) + ": " + hipGetErrorString(_e)};           \
    } while (0)

// The thread-local message behind hg_last_error (api.cpp).
std::string& last_error_ref();
inline hg_status fail(hg_status code, const std::string& msg) {
    last_error_ref() = msg;
    return code;
}
// Runs an entry point's body, converting exceptions to status codes.
template <class F>
hg_status guarded(F&& fn) {
    try {
        last_error_ref().clear();
        return fn();
    } catch (const Error& e) {
        return fail(e.code, e.msg);
    } catch (const std::bad_alloc&) {
        return fail(HG_E_OOM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(HG_E_DEVICE, e.what());
    } catch (...) {
        return fail(HG_E_DEVICE, "unknown error");
    }
}

// A device buffer owned by the library.
template <class T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    void alloc(size_t count) {
        if (count == n && p) return;
        release();
        if (count == 0) return;
        HG_CHECK_HIP(hipMalloc(&p, count * sizeof(T)));
        n = count;
    }
    void upload(const std::vector<T>& h, hipStream_t s) {
        alloc(h.size());
        if (!h.empty())
            HG_CHECK_HIP(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    }
    size_t bytes() const { return n * sizeof(T); }
};

// Face slot encoding: slot (f, k) refers to the edge (tri[k], tri[k+1]):
//   fslot = (edge << 2) | (boundary << 1) | side,
// side = which of the edge's two incident faces f is (0 or 1).
__host__ __device__ inline int slot_edge(uint32_t s) { return (int)(s >> 2); }
__host__ __device__ inline int slot_side(uint32_t s) { return (int)(s & 1u); }
__host__ __device__ inline int slot_bnd(uint32_t s) { return (int)((s >> 1) & 1u); }

// Host-side topology produced by build_topology().
struct HostTopo {
    int64_t nv = 0, nf = 0, ne = 0, nbnd = 0;
    int max_valence = 0;
    std::vector<int32_t> perm_v, iperm_v;   // internal -> caller, caller -> internal
    std::vector<double> px, py, pz;         // positions, internal order
    std::vector<int32_t> row_ptr, col, csr_edge;
    std::vector<int32_t> tri;               // [nf*3] internal vertex ids
    std::vector<int32_t> perm_f;            // internal face -> caller face
    std::vector<uint32_t> fslot;            // [nf*3]
    std::vector<uint8_t> fsign;             // bit k: slot k has sign +1 (Eq. 20)
    std::vector<int32_t> ev;                // [ne*2] tail, head (internal ids)
    std::vector<int32_t> ef;                // [ne*2] incident faces, -1 if none
    std::vector<int32_t> perm_e;            // internal edge -> canonical edge
    std::vector<int32_t> twin, h01;         // per slot: the other face's slot (-1); per edge: its two slots
    // tiles (contiguous internal vertex ranges) and their halos
    int patch_size = 0;
    std::vector<int32_t> tile_ptr;          // [n_tiles+1] first internal vertex
    std::vector<int32_t> halo_ptr, halo_idx;
    std::vector<uint16_t> lnb;              // ELL local neighbour slots
    std::vector<int32_t> ell_ptr;           // per patch: offset of its ELL block
    std::vector<uint8_t> ell_width;         // per patch: ELL width
    // colouring of the tile adjacency graph (tiles sharing a mesh edge get
    // different colours): tiles of colour c are tile_order[color_ptr[c] ..]
    std::vector<int32_t> color_ptr, tile_order;
    // the tile adjacency itself (CSR, neighbours ascending)
    std::vector<int32_t> tile_adj_ptr, tile_adj;
    // connected components: comp[v] per internal vertex, numbered in the
    // order of their smallest caller vertex id; mean edge length of each;
    // the component of each tile (tiles are connected)
    int n_comp = 0;
    std::vector<int32_t> comp, tile_comp;
    std::vector<double> comp_hbar;
    int max_halo = 0;
    int max_ell_width = 0;
    // generator loops of closed components of genus > 0 (Sec. 5.1), see
    // build_cycles: edge loops (internal edge, sign) and face loops
    // (internal face, the edge the loop leaves it by, polyline segment);
    // cyc_e_face: a face of each edge-loop slot's edge; cyc_e_canon,
    // cyc_f_caller: the caller's ids of the loops' edges and faces
    int n_cycles = 0;
    std::vector<int32_t> cyc_e_ptr, cyc_e_edge, cyc_e_face, cyc_f_ptr, cyc_f_face, cyc_f_edge;
    std::vector<int32_t> cyc_e_canon, cyc_f_caller;
    std::vector<float> cyc_e_sign, cyc_f_vec;
};

// Builds the host topology; throws Error{HG_E_BAD_MESH} on invalid input.
// slots > 0: the tile colours are balanced for launches that run that many
// tile workgroups at a time (see colour_tiles).
void build_topology(const double* xyz, int64_t nv, const int32_t* tri, int64_t nf, int patch_size,
                    HostTopo& out, int slots = 0);
// Fills the cyc_* loops of a built topology (tree-cotree, caller-id rules).
void build_cycles(HostTopo& T);
// Colours of a conflict graph (symmetric adjacency lists, no self loops) by
// saturation-degree ordering: fewer colours than greedy in index order (five
// instead of six on the icosphere tiles).  With slots > 0 (the workgroups a
// colour's launch runs at a time) a colour of n nodes takes ceil(n / slots)
// waves, so nodes just past a multiple of slots are moved, where no
// neighbour has the target colour, to colours with room below their next
// multiple.  Fills color_ptr [ncol+1] and order (the nodes grouped by
// colour, ascending within a colour).
void colour_tiles(const std::vector<std::vector<int32_t>>& adj, std::vector<int32_t>& color_ptr,
                  std::vector<int32_t>& order, int slots = 0);

// Intrinsic Delaunay triangulation (edge flips on intrinsic lengths) of a
// caller mesh: the flipped triangles (caller vertex ids, rows in the input's
// order) and the length of every edge of the result.
struct EdgeTable {   // edge key (min id << 32 | max id) -> record, open addressing
    static constexpr uint64_t kEmpty = ~0ull, kTomb = ~0ull - 1;
    std::vector<uint64_t> key;
    std::vector<int32_t> val;
    size_t used = 0, tomb = 0;
    void init(size_t n_keys);
    size_t slot_of(uint64_t k) const;
    int32_t find(uint64_t k) const;   // -1 if absent
    void insert(uint64_t k, int32_t v);
    void erase(uint64_t k);
    void rehash();
};
struct IntrinsicTri {
    std::vector<int32_t> tri;
    EdgeTable index;                               // edge -> record
    std::vector<double> rec_len;                   // length per record
    int64_t n_flips = 0, n_nondelaunay = 0;
    double hbar_input = 0.0;                       // mean edge length of the input mesh
    std::vector<int32_t> input_a;                  // input edges: one endpoint and the length
    std::vector<double> input_len;
    double edge_length(int32_t a, int32_t b) const;
};
void build_intrinsic(const double* xyz, int64_t nv, const int32_t* tri, int64_t nf, IntrinsicTri& out);

// Face tiles with halos for the blocked edge-ADMM launch (admm_tiles.cpp):
// tile p owns faces [f0[p], f0[p+1]); its region is those faces followed by
// the halo faces halo[rptr[p] - f0[p] ..] up to `rings` edge-adjacency steps
// away; rec[rptr[p] + r] is region face r's record (twin copies, signs).
constexpr int kMaxAdmmBlock = 8;    // iterations per blocked launch at most
constexpr int kAutoAdmmBlock = 6;   // hg_opts.admm_block = 0
constexpr int kAutoOverlapRings = 2; // hg_opts.overlap_rings = 0
constexpr uint32_t kTwinNone = 0xFFFF;   // boundary slot: no twin
constexpr uint32_t kTwinOut = 0xFFFE;    // twin outside the region
struct EdgeTiles {
    int rings = 0, max_region = 0;
    std::vector<int32_t> f0, rptr, halo;
    std::vector<uint64_t> rec;
};
// false if a region would exceed max_region faces or the faces are not in
// tile order
bool build_edge_tiles(int64_t nf, const std::vector<int32_t>& tri, const std::vector<int32_t>& twin,
                      const std::vector<uint8_t>& fsign, const std::vector<int32_t>& tile_ptr, int rings,
                      int max_region, EdgeTiles& out);

// Overlapping diffusion tiles (overlap_tiles.cpp): per tile, halo_idx holds
// its n_ov overlap vertices (updated by the in-tile sweeps, never written
// back) followed by the fixed outer ring; ELL rows of the core (stride P)
// then of the overlap vertices (stride n_ov); colours such that no tile
// reads the core of a tile of its own colour.
struct OverlapTiles {
    int rings = 0, max_halo = 0, max_ov = 0, max_ell_width = 0;
    std::vector<int32_t> halo_ptr, halo_idx, n_ov, ell_ptr, color_ptr, tile_order;
    std::vector<uint8_t> ell_width;
    std::vector<uint16_t> lnb;
};
// A tile whose region with `rings` rings would exceed lds_budget bytes
// (values, exponents and, per overlap vertex, lds_width coefficients and
// slots) or max_ov overlap vertices gets fewer rings.  false if even the
// plain halo leaves too many overlap vertices or the region does not fit
// 16-bit local slots.
bool build_overlap_tiles(const std::vector<int32_t>& row_ptr, const std::vector<int32_t>& col,
                         const std::vector<int32_t>& tile_ptr, int P, int rings, int max_ov, OverlapTiles& out,
                         size_t lds_budget = ~(size_t)0, int lds_width = 16);

// Per-query device workspace.  A query runs on one Work and one stream; the
// mesh data it reads is never written after mesh_create, so queries on the
// same mesh with different Works may run concurrently on different streams.
// Buffers grow on demand and are kept for the next query.
struct Work {
    Work() = default;
    Work(const Work&) = delete;
    Work& operator=(const Work&) = delete;
    ~Work() {
        if (pinned) (void)hipHostFree(pinned);
        if (ev) (void)hipEventDestroy(ev);
        if (own_stream) (void)hipStreamDestroy(own_stream);
    }
    void ensure_pinned() {
        if (!pinned) HG_CHECK_HIP(hipHostMalloc(&pinned, 8 * sizeof(double), hipHostMallocDefault));
    }
    // a stream of the workspace's own (default priority, non-blocking), used
    // in place of the null stream, which cannot be captured into a graph
    hipStream_t own_stream = nullptr;
    hipEvent_t ev = nullptr;
    void ensure_stream() {
        if (!own_stream) HG_CHECK_HIP(hipStreamCreateWithFlags(&own_stream, hipStreamNonBlocking));
        if (!ev) HG_CHECK_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    }
    DBuf<int32_t> level, parent, pedge, frontier_a, frontier_b, counters;   // pedge: the edge to the parent
    DBuf<double> v0, v1, invD;          // diffusion mantissas, 1/(A + t sum theta)
    DBuf<double> tcomp, tile_t;         // diffusion time per component and per tile
    DBuf<int32_t> e0, e1;               // diffusion exponents
    DBuf<double> logu;
    DBuf<float> h;                      // [nf*3] internal order; the edge form reads it only
                                        // for the targets and then keeps the blocked ADMM's
                                        // state one iteration back in it
    DBuf<float> sumz;                   // [ne] edge-form target sums
    DBuf<float> sumd;                   // [3nf] target sum of each slot's edge
    DBuf<float> z0, z1;                 // edge form: zeta [3*nf]; face form: z [9*nf]
    DBuf<float> g0, g1;                 // face form gradients [nf*3]
    DBuf<float> xe;                     // [ne] final edge differences (internal)
    DBuf<float> gf;                     // [nf*3] final face gradients (internal)
    DBuf<float> shi0, slo0, shi1, slo1; // integration double-float sums
    DBuf<int32_t> jp0, jp1;             // pointer-jumping parents
    DBuf<float> dprev;                  // distance at the previous ADMM check
    DBuf<double> comp_pair;             // per component (largest change, largest d) of a check
    DBuf<int32_t> tile_mark;            // tiled search: last pass a tile or a neighbour changed
    DBuf<uint8_t> tile_on, cflag;       // ADMM tiles still iterating; per component 0 active,
                                        // 1 stopping now, 2 stopped
    DBuf<uint8_t> cdue, bdue;           // per component: checked now; per vertex block of a
                                        // check: 0 none, 1 all, 2 some of its vertices checked
    DBuf<double> partial;               // reduction partials
    DBuf<double> red_host_dummy;
    double* pinned = nullptr;           // host pinned reduction results
    DBuf<int32_t> src;
    // conjugate gradients of the Sec. 6.4 comparator (kernels_cg.hip)
    struct Cg {
        DBuf<double> x, r, z, p, q, D, b, partial, scal;
        DBuf<uint8_t> fixed;
        size_t bytes() const {
            return x.bytes() + r.bytes() + z.bytes() + p.bytes() + q.bytes() + D.bytes() + b.bytes() +
                   partial.bytes() + scal.bytes() + fixed.bytes();
        }
    } cg;
    // source paths of the multi-source constraints (Eqs. 24-25), built by
    // build_source_paths: np paths over ns slots, slots grouped by edge
    // and by face (CSR over the distinct ids, slots in increasing order)
    struct Paths {
        int np = 0, ns = 0, ng_edge = 0, ng_face = 0;
        int np_src = 0, ns_src = 0;             // the source paths: groups [0, np_src), slots [0, ns_src)
        int n_cyc = 0, ns_cyc = 0;              // the generator loops after them
        int max_len = 0;                        // slots of the longest group
        int max_len_src = 0, max_len_cyc = 0;   // of the longest source path / generator loop
        DBuf<int32_t> ptr, edge, face;
        DBuf<float> sign, vec;                  // [ns], [3*ns]
        DBuf<int32_t> eg_ptr, eg_id, eg_slot, fg_ptr, fg_id, fg_slot;
        DBuf<int2> zslot;                       // per path slot: the edge's two face slots (edge form)
        DBuf<int2> gzslot;                      // per edge group: the same
        DBuf<float> z;                          // folded copies: [ns] edge form, [3*ns] face form
        DBuf<float> seff;                       // edge form: [ne] effective target sums
        // each group's slots cut into chunks of kPathChunk; a chunk's
        // partial sums of the projection, the group of each slot
        int nch = 0;
        DBuf<int32_t> spath, cptr, chunk_path;  // [ns], [np+1], [nch]
        DBuf<double> pc;                        // [2 nch]
        size_t bytes() const;
    } paths;
    size_t bytes() const;
};

struct Mesh {
    int device = 0;
    int64_t nv = 0, nf = 0, ne = 0, nbnd = 0;
    int max_valence = 0;
    double hbar = 0.0, total_area = 0.0;
    std::vector<int32_t> iperm_v_host;      // caller id -> internal id (host copy)

    DBuf<double> px, py, pz;
    DBuf<int32_t> perm_v, perm_f, perm_e;
    DBuf<int32_t> row_ptr, col, csr_edge;
    DBuf<double> theta;                     // per CSR entry
    DBuf<double> Av, sum_theta;             // per vertex
    DBuf<int32_t> tri;
    DBuf<uint32_t> fslot;
    DBuf<uint8_t> fsign;
    DBuf<double> farea;                     // per face (FP64)
    DBuf<int32_t> ev, ef;
    // face form only, built by the first face-form iteration (ensure_sgeo):
    // per face slot the unit edge vector and A_nb / (A_own + A_nb)
    DBuf<float4> sgeo;
    mutable std::mutex sgeo_mu;
    DBuf<int32_t> twin, h01;
    // edge form, blocked launches: face tiles with halos, one set per halo
    // depth used, built by the first blocked iteration with that depth
    // (ensure_edge_tiles) and kept until the mesh is destroyed, so that
    // concurrent queries never see a set replaced
    struct EdgeTileSet {
        int rings = 0, max_region = 0, n = 0;
        bool ok = false;   // false: a region does not fit in LDS
        DBuf<int32_t> f0, rptr, halo;
        DBuf<uint64_t> rec;
    };
    std::vector<std::unique_ptr<EdgeTileSet>> etiles;
    mutable std::mutex et_mu;
    // diffusion tiles with `rings` rings of overlap (OverlapTiles on the
    // device), one set per depth used, built on first use and kept
    struct OverlapTileSet {
        int rings = 0, max_halo = 0, max_ov = 0, max_ell_width = 0;
        bool ok = false;
        DBuf<int32_t> halo_ptr, halo_idx, n_ov, ell_ptr, tile_order;
        DBuf<uint8_t> ell_width;
        DBuf<uint16_t> lnb;
        std::vector<int32_t> color_ptr_host;
        size_t bytes() const {
            return halo_ptr.bytes() + halo_idx.bytes() + n_ov.bytes() + ell_ptr.bytes() + tile_order.bytes() +
                   ell_width.bytes() + lnb.bytes();
        }
    };
    std::vector<std::unique_ptr<OverlapTileSet>> otiles;
    mutable std::mutex ot_mu;

    // patch tiles
    int patch_size = 0, n_patches = 0, max_halo = 0, max_ell_width = 0;
    DBuf<int32_t> tile_ptr, halo_ptr, halo_idx, ell_ptr;
    DBuf<int32_t> tile_k0;                  // [n_tiles+1] first CSR entry of each tile's rows
    DBuf<int32_t> tile_adj_ptr, tile_adj;   // tile adjacency (HostTopo)
    DBuf<uint16_t> lnb;
    DBuf<uint8_t> ell_width;
    std::vector<int32_t> color_ptr_host;    // tile colours (see HostTopo)
    DBuf<int32_t> tile_order;
    // connected components (see HostTopo)
    int n_comp = 0;
    std::vector<double> comp_hbar_host;
    DBuf<int32_t> comp_v, tile_comp;

    // generator loops of closed components of genus > 0 (host copies of
    // HostTopo's cyc_*), added to a query's constraint groups
    int n_cycles = 0;
    std::vector<int32_t> cyc_e_ptr, cyc_e_edge, cyc_e_face, cyc_f_ptr, cyc_f_face, cyc_f_edge;
    std::vector<int32_t> cyc_e_canon, cyc_f_caller;
    std::vector<float> cyc_e_sign, cyc_f_vec;

    // intrinsic triangulation (hg_mesh_create_intrinsic): the faces are the
    // flipped ones, floc[3f..3f+2] = (l_01, x_2, y_2) places face f's corners
    // at (0, 0), (l_01, 0), (x_2, y_2) in its own plane; gradients and edge
    // targets are taken in these frames
    bool intrinsic = false;
    int64_t n_flips = 0, n_nondelaunay = 0;
    DBuf<double> floc;
    std::vector<int32_t> idt_tri_host;                // caller vertex ids, [nf*3]
    std::vector<double> idt_len_canon;                // per canonical edge

    // diffusion schedule picked by hg_mesh_autotune for options left at 0
    // (auto): 0 = not tuned
    int tuned_schedule = 0, tuned_inner = 0, tuned_rings = 0, tuned_admm_block = 0;
    // default per-query workspace of the synchronous entry points (also
    // used for the mesh's own reductions)
    Work w;

    uint64_t mesh_bytes() const;
    void ensure_sgeo(hipStream_t s);
    // the blocked edge-ADMM tiles for `rings` (nullptr if the mesh's regions
    // do not fit in LDS)
    const EdgeTileSet* ensure_edge_tiles(int rings, hipStream_t s);
    // the overlapping diffusion tiles for `rings` (nullptr if a tile has more
    // than max_ov overlap vertices)
    const OverlapTileSet* ensure_overlap_tiles(int rings, int max_ov, size_t lds_budget, int lds_width,
                                               hipStream_t s);
    ~Mesh();
};

// ---- kernels / stage drivers (implemented in the .hip files) ----
// elen: per internal edge length (intrinsic meshes; positions otherwise)
void geometry_init(Mesh& m, hipStream_t s, const std::vector<double>* elen = nullptr);
int run_bfs(Mesh& m, Work& w, const std::vector<int32_t>& src_internal, hipStream_t s);
// The breadth-first search on caller-provided device buffers: level, parent,
// pedge (the edge to the parent), frontier_a, frontier_b [nv] each, counters [8],
// src [nsrc].
struct BfsBuffers {
    int32_t *level, *parent, *pedge, *frontier_a, *frontier_b, *counters, *src;
};
int run_bfs_into(Mesh& m, const BfsBuffers& b, const std::vector<int32_t>& src_internal, hipStream_t s);
// caller id -> internal id of each source, checked (throws HG_E_INVALID_ARG)
std::vector<int32_t> map_sources(const Mesh& m, const int32_t* src, int32_t nsrc);
struct DiffusionResult {
    int sweeps = 0, passes = 0;
    double res = 0.0;
    bool converged = false;
    double kernel_ms = 0.0;      // summed event time of the pass kernels
    int timed_launches = 0;      // launches covered by kernel_ms
    uint64_t bytes_per_pass = 0; // algorithmic HBM bytes of one pass kernel
};
// t[c]: diffusion time of component c (one entry per connected component)
DiffusionResult run_diffusion(Mesh& m, Work& w, const std::vector<int32_t>& src_internal,
                              const std::vector<double>& t,
                              const hg_opts& o, hipStream_t s);
void diffusion_logu(Mesh& m, Work& w, hipStream_t s);                   // w.logu from (v, e)
bool patch_supported(const Mesh& m);
// overlap > 0: the overlapping tiles with that many rings
DiffusionResult run_diffusion_patch(Mesh& m, Work& w, const hg_opts& o, int inner, hipStream_t s, int overlap = 0);
void run_normalize(Mesh& m, Work& w, hipStream_t s);                    // w.h from (v, e)
void normalize_from_logu(Mesh& m, Work& w, const double* logu_user, hipStream_t s);
struct AdmmResult {
    int iters = 0;
    double rp = 0.0, rd = 0.0;
    double seam = 0.0;           // last check's largest seam / hbar (distance monitor only)
    bool converged = false;
    double kernel_ms = 0.0;
    int timed_launches = 0;
    uint64_t bytes_per_iter = 0;  // algorithmic bytes of one launch of the main kernel
    int launches = 0;             // launches of the main kernel (blocked: several iterations each)
    int block = 1;                // iterations per launch of the main kernel
};

// Events around runs of back-to-back launches of one kernel (between two
// convergence checks) give its average device time without per-launch events.
struct RunTimer {
    hipEvent_t a = nullptr, b = nullptr;
    bool open = false;
    RunTimer() {
        HG_CHECK_HIP(hipEventCreate(&a));
        HG_CHECK_HIP(hipEventCreate(&b));
    }
    ~RunTimer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    void start(hipStream_t s) {
        HG_CHECK_HIP(hipEventRecord(a, s));
        open = true;
    }
    // closes the run; the caller synchronises the stream before reading
    double stop(hipStream_t s) {
        if (!open) return 0.0;
        HG_CHECK_HIP(hipEventRecord(b, s));
        HG_CHECK_HIP(hipEventSynchronize(b));
        float ms = 0.f;
        HG_CHECK_HIP(hipEventElapsedTime(&ms, a, b));
        open = false;
        return ms;
    }
};
// A fixed sequence of launches captured once into a HIP graph and replayed
// (one graph launch instead of many kernel launches).  Only kernel launches
// are captured.  capture() returns false (and the caller runs the launches
// directly) where the stream cannot be captured.
struct GraphChunk {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    bool tried = false;
    GraphChunk() = default;
    GraphChunk(const GraphChunk&) = delete;
    GraphChunk& operator=(const GraphChunk&) = delete;
    ~GraphChunk() {
        if (x) (void)hipGraphExecDestroy(x);
        if (g) (void)hipGraphDestroy(g);
    }
    template <class F>
    bool capture(hipStream_t s, F&& enqueue) {
        tried = true;
        if (!s) return false;
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
        enqueue();
        hipGraph_t gg = nullptr;
        const hipError_t e = hipStreamEndCapture(s, &gg);
        if (e != hipSuccess || !gg) {
            (void)hipGetLastError();
            return false;
        }
        g = gg;
        if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGetLastError();
            x = nullptr;
            return false;
        }
        return true;
    }
    bool ready() const { return x != nullptr; }
    void launch(hipStream_t s) { HG_CHECK_HIP(hipGraphLaunch(x, s)); }
};

// iters > 0: exactly that many iterations.  Otherwise run to convergence:
// with depth >= 0 (the breadth-first depth of the query) by the change of the
// integrated distance field (DistStop), else by the paper's residuals.
// With use_paths, the constraints of Eqs. 24-25 over m.w.paths are added.
AdmmResult run_admm_edge(Mesh& m, Work& w, int iters, const hg_opts& o, hipStream_t s, int depth = -1,
                         bool use_paths = false);
AdmmResult run_admm_face(Mesh& m, Work& w, int iters, const hg_opts& o, hipStream_t s, int depth = -1,
                         bool use_paths = false);
// Builds w.paths: with source_paths, the paths between the (internal)
// sources (Eqs. 24-25); with cycles, the mesh's generator loops in the given
// form (Sec. 5.1).  The source paths come from breadth-first searches from
// single sources, which overwrite level/parent/pedge: run the query's own
// breadth-first search after it.
void build_constraint_paths(Mesh& m, Work& w, const std::vector<int32_t>& src_internal, bool source_paths,
                            bool cycles, int form, hipStream_t s);
void integrate(Mesh& m, Work& w, int form, int depth, float* d_user, hipStream_t s);
// The edge-form state an edge difference is formed from (Eq. 21):
// x_e = (S_e + zeta_h0 + zeta_h1) / (|H_e| (1 + mu)), a boundary edge without
// zeta_h1.  Given to the distance checks, which then form x only on the
// edges the integration follows instead of reading a full x array.
struct EdgeX {
    const float* S;
    const float* z;
    float inv1mu;
};
__device__ inline float edge_x(float S, float z0, float z1, int bnd, float inv1mu) {
    // x_e = (S + z0 + z1) / (|H_e| (1 + mu)); a boundary edge has z1 = 0
    return bnd ? (S + z0) * inv1mu : 0.5f * (S + z0 + z1) * inv1mu;
}
// integrates the given state (edge differences xe or face gradients g) and
// returns max |d - d_prev| (inf on the first call) and max |d|; d_prev <- d;
// with seam, also the largest |d_head - d_tail - x_e| over the edges
void dist_change(Mesh& m, Work& w, int form, int depth, const float* xe, const float* g, bool first, hipStream_t s,
                 double& delta, double& dmax, double* seam = nullptr, const EdgeX* ex = nullptr);
// the largest |d_head - d_tail - x_e| for the d of the last dist_change and
// the given field (the same state)
double seam_now(Mesh& m, Work& w, int form, const float* xe, const float* g, hipStream_t s);
// As dist_change, per connected component (delta[c], dmax[c]).  With due
// (host, one byte per component), only the components with due[c] != 0 are
// integrated and compared (the others keep their d_prev, and their delta and
// dmax come back 0).
void dist_change_comp(Mesh& m, Work& w, int form, int depth, const float* xe, const float* g, bool first,
                      hipStream_t s, std::vector<double>& delta, std::vector<double>& dmax, const EdgeX* ex = nullptr,
                      const uint8_t* due = nullptr);

// Stopping rule on the distance field: with delta_k the largest change of d
// between two checks and r = delta_k / delta_{k-1} < 1, the remaining change
// of a geometrically converging iteration is at most delta_k r / (1 - r);
// stop once that is <= tol * max|d|, or once delta_k itself is at the FP32
// rounding floor (<= tol * max|d| / 100; the rounding noise of d is orders of
// magnitude lower, and a slowly converging iteration -- time constant tau
// iterations -- is only stopped early by this rule if tau >~ 64 * 100).
//
// Checks run every chunk of iterations; while the estimated remaining change
// is far above the tolerance (> 300 tol max|d|) they run every
// kCoarseChecks chunks instead, back to every chunk once it is within
// 30 tol max|d|.  restart() drops the ratio at a switch, so that a decision
// always compares two intervals of the same length.
struct DistStop {
    bool first = true;
    double prev = 0.0;
    double est = INFINITY;   // last estimate of the remaining change
    bool update(double delta, double dmax, double tol) {
        bool done = false;
        est = INFINITY;
        if (!first && std::isfinite(delta)) {
            if (std::isfinite(prev) && prev > 0.0 && delta < prev) {
                double r = delta / prev;
                est = delta * r / (1.0 - r);
                done = est <= tol * dmax;
            }
            if (delta <= 0.01 * tol * dmax) done = true;
        }
        first = false;
        prev = delta;
        return done;
    }
    bool near(double dmax, double tol) const { return est <= 30.0 * tol * dmax; }
    bool far(double dmax, double tol) const { return std::isfinite(est) && est > 300.0 * tol * dmax; }
    void restart() { prev = NAN; }
};
constexpr int kCoarseChecks = 4;   // chunks between checks far from convergence

// One whole query (the body of hg_geodesic_solve) on a given workspace and
// stream; throws Error for invalid arguments and device failures.
struct QueryOutcome {
    hg_status status;
    std::string msg;
};
QueryOutcome solve_query(Mesh& m, Work& w, const int32_t* src, int32_t nsrc, double t, const hg_opts* opts,
                         float* d_dev, hipStream_t s, hg_info* info);

// The join of several resident meshes as the components of one mesh (device
// arrays concatenated with shifted indices; batch.cpp), and the release of a
// cached join that holds a mesh about to be destroyed.
std::unique_ptr<Mesh> join_meshes(const std::vector<Mesh*>& parts, hipStream_t s);
void forget_joins_with(Mesh* m);
// Upper estimate of the device bytes of one query's workspace (server.cpp).
uint64_t work_estimate(const Mesh& m, int form, int nsrc);

// Conjugate gradients with a diagonal preconditioner (Sec. 6.4) on the heat
// system (op 0), the face-form Poisson system (1) or the edge-form one (2);
// the result is in w.cg.x (internal order).  tol > 0: stop at relative
// residual <= tol (checked every 16 iterations); tol = 0: max_iters exactly.
struct CgResult {
    int iters = 0;
    bool converged = false;
    double res_rel = 0.0, res_abs = 0.0, res_abs0 = 0.0, ms = 0.0;
};
CgResult run_cg(Mesh& m, Work& w, int op, const std::vector<int32_t>& src_internal, const std::vector<double>& tc,
                const float* h_internal, int max_iters, double tol, hipStream_t s);
// |(A - t L_c) u - u_0|_2 (Sec. 6.4's E_1) for u in internal order (log u if is_log)
double heat_residual(Mesh& m, Work& w, const std::vector<int32_t>& src_internal, const std::vector<double>& tc,
                     const double* u_internal, bool is_log, hipStream_t s);

// permutation helpers
void gather_faces_to_internal(Mesh& m, const float* user3, float* internal3, hipStream_t s);
void scatter_faces_to_user(Mesh& m, const float* internal3, float* user3, hipStream_t s);
void scatter_edges_to_user(Mesh& m, const float* internal, float* user, hipStream_t s);
void gather_edges_to_internal(Mesh& m, const float* user, float* internal, hipStream_t s);
void scatter_vertices_to_user_d(Mesh& m, const double* internal, double* user, hipStream_t s);
void gather_vertices_to_internal_d(Mesh& m, const double* user, double* internal, hipStream_t s);
void scatter_vertices_to_user_i(Mesh& m, const int32_t* internal, int32_t* user, bool map_values,
                                hipStream_t s);
void edges_to_user(Mesh& m, int32_t* edges_user, hipStream_t s);
void weights_to_user(Mesh& m, double* theta_user, double* area_user, hipStream_t s);

// reductions: sum or max of n doubles produced per block into w.partial
double reduce_partials(Mesh& m, Work& w, int nblocks, bool is_max, hipStream_t s);

inline int grid_for(int64_t n, int block) { return (int)((n + block - 1) / block); }

// slots of a constraint group summed by one workgroup of the edge-form
// projection (several workgroups per long path or loop)
constexpr int kPathChunk = 1024;

// Blocks are dealt round-robin to the 8 XCDs of an MI355X; remap so that
// each XCD processes one contiguous range of the index space (consecutive
// blocks share halo cache lines in that XCD's L2).
__device__ inline int xcd_block(int b, int nb) {
    const int nx = 8;
    int per = nb / nx, rem = nb % nx;
    int x = b % nx, i = b / nx;
    int start = x * per + (x < rem ? x : rem);
    int idx = start + i;
    return idx;
}

}  // namespace hg
