// hg_bfs_noalloc: the breadth-first search of hg_bfs on a fixed device
// array of the library instead of buffers it allocates, for callers that
// cannot allocate device memory.
//
// `scratch` holds the search's working arrays (internal-order levels,
// parents and pairing slots, the two frontier queues, the counters and the
// source list).  Each GPU that runs this entry point holds its own copy of
// the array until the process ends.  Host code never passes the array's name
// to a kernel or a copy (on the host it is only a stand-in for the symbol):
// its device address is looked up once per device with hipGetSymbolAddress
// and that address is used everywhere.  Every call on one GPU shares that
// GPU's array and leaves the last call's contents in it; the search clears
// what must start cleared (levels, counters) itself.  Calls that overlap on
// one GPU race on the array.
#include <mutex>

#include "hgeo_internal.h"

namespace hg {

constexpr size_t kScratchBytes = 64ull << 20;      // 64 MiB per device
constexpr int64_t kNoallocMaxV = 3000000;          // 5 int32 arrays of nv
constexpr int32_t kNoallocMaxSrc = 65536;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_dev[64];   // device address of `scratch` per device id

// The device address of this device's `scratch` (looked up on first use).
static unsigned char* scratch_on(int dev) {
    if (dev < 0 || dev >= 64) throw Error{HG_E_DEVICE, "device id out of range"};
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            throw Error{HG_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
        g_scratch_dev[dev] = p;
    }
    return static_cast<unsigned char*>(g_scratch_dev[dev]);
}

static size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

}  // namespace hg

using namespace hg;

extern "C" hg_status hg_bfs_noalloc(hg_mesh_t mesh, const int32_t* src, int32_t nsrc, int32_t* level_dev,
                                    int32_t* parent_dev, void* stream, int32_t* depth_out) {
    return guarded([&]() -> hg_status {
        if (!mesh) return fail(HG_E_INVALID_ARG, "null mesh");
        auto* m = reinterpret_cast<Mesh*>(mesh);
        if (m->nv > kNoallocMaxV)
            return fail(HG_E_INVALID_ARG, "hg_bfs_noalloc: mesh has " + std::to_string(m->nv) +
                                              " vertices, more than the limit of " + std::to_string(kNoallocMaxV));
        if (nsrc > kNoallocMaxSrc)
            return fail(HG_E_INVALID_ARG, "hg_bfs_noalloc: more than " + std::to_string(kNoallocMaxSrc) +
                                              " sources");
        int dev = -1;
        HG_CHECK_HIP(hipGetDevice(&dev));
        if (dev != m->device) return fail(HG_E_INVALID_ARG, "hg_bfs_noalloc: the mesh lives on another device");
        auto si = map_sources(*m, src, nsrc);
        // carve the arrays out of this device's scratch
        const size_t nvb = align256((size_t)m->nv * sizeof(int32_t));
        const size_t need = 5 * nvb + 256 + align256((size_t)nsrc * sizeof(int32_t));
        if (need > kScratchBytes) return fail(HG_E_INVALID_ARG, "hg_bfs_noalloc: scratch too small");
        unsigned char* base = scratch_on(dev);
        auto take = [&](size_t bytes) {
            int32_t* p = reinterpret_cast<int32_t*>(base);
            base += bytes;
            return p;
        };
        BfsBuffers b;
        b.level = take(nvb);
        b.parent = take(nvb);
        b.pedge = take(nvb);
        b.frontier_a = take(nvb);
        b.frontier_b = take(nvb);
        b.counters = take(256);
        b.src = take(align256((size_t)nsrc * sizeof(int32_t)));
        hipStream_t s = (hipStream_t)stream;
        const int depth = run_bfs_into(*m, b, si, s);
        if (level_dev) scatter_vertices_to_user_i(*m, b.level, level_dev, false, s);
        if (parent_dev) scatter_vertices_to_user_i(*m, b.parent, parent_dev, true, s);
        HG_CHECK_HIP(hipStreamSynchronize(s));
        if (depth_out) *depth_out = depth;
        return HG_OK;
    });
}
