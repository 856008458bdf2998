// C ABI of the hgeo library (declared in include/hgeo.h): argument checks,
// conversion of errors to status codes, and the order of the stages of one
// solve (Algorithm 1 of the paper).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "hgeo_internal.h"

namespace hg {

static thread_local std::string g_last_error;
std::string& last_error_ref() { return g_last_error; }

size_t Work::bytes() const {
    return level.bytes() + parent.bytes() + pedge.bytes() + frontier_a.bytes() + frontier_b.bytes() +
           counters.bytes() + v0.bytes() + v1.bytes() + invD.bytes() + e0.bytes() + e1.bytes() + logu.bytes() +
           h.bytes() + sumz.bytes() + sumd.bytes() + z0.bytes() + z1.bytes() + g0.bytes() + g1.bytes() + xe.bytes() + gf.bytes() +
           shi0.bytes() + slo0.bytes() + shi1.bytes() + slo1.bytes() + jp0.bytes() + jp1.bytes() + partial.bytes() +
           src.bytes() + dprev.bytes() + comp_pair.bytes() + tile_mark.bytes() + tile_on.bytes() + cflag.bytes() +
           cdue.bytes() + bdue.bytes() +
           paths.bytes() +
           tcomp.bytes() + tile_t.bytes() + cg.bytes();
}

size_t Work::Paths::bytes() const {
    return ptr.bytes() + edge.bytes() + face.bytes() + sign.bytes() + vec.bytes() + eg_ptr.bytes() + eg_id.bytes() +
           eg_slot.bytes() + fg_ptr.bytes() + fg_id.bytes() + fg_slot.bytes() + z.bytes() + seff.bytes() +
           zslot.bytes() + gzslot.bytes();
}

uint64_t Mesh::mesh_bytes() const {
    uint64_t face_form = 0;
    {
        std::lock_guard<std::mutex> lock(sgeo_mu);
        face_form = sgeo.bytes();
    }
    uint64_t blocked = 0;
    {
        std::lock_guard<std::mutex> lock(et_mu);
        for (const auto& t : etiles) blocked += t->f0.bytes() + t->rptr.bytes() + t->halo.bytes() + t->rec.bytes();
    }
    {
        std::lock_guard<std::mutex> lock(ot_mu);
        for (const auto& t : otiles) blocked += t->bytes();
    }
    return face_form + blocked + floc.bytes() + px.bytes() + py.bytes() + pz.bytes() + perm_v.bytes() + perm_f.bytes() + perm_e.bytes() +
           row_ptr.bytes() + col.bytes() + csr_edge.bytes() + theta.bytes() + Av.bytes() + sum_theta.bytes() +
           tri.bytes() + fslot.bytes() + fsign.bytes() + farea.bytes() + ev.bytes() + ef.bytes() +
           tile_ptr.bytes() + tile_k0.bytes() + tile_adj_ptr.bytes() + tile_adj.bytes() + halo_ptr.bytes() + halo_idx.bytes() + ell_ptr.bytes() + lnb.bytes() + ell_width.bytes() +
           tile_order.bytes() + twin.bytes() + h01.bytes() + comp_v.bytes() + tile_comp.bytes();
}

Mesh::~Mesh() = default;


std::vector<int32_t> map_sources(const Mesh& m, const int32_t* src, int32_t nsrc) {
    if (!src || nsrc <= 0) throw Error{HG_E_INVALID_ARG, "empty source list"};
    std::vector<int32_t> out;
    out.reserve(nsrc);
    for (int32_t i = 0; i < nsrc; ++i) {
        if (src[i] < 0 || src[i] >= m.nv) throw Error{HG_E_INVALID_ARG, "source index out of range"};
        out.push_back(m.iperm_v_host[src[i]]);
    }
    return out;
}

static hg_opts resolve_opts(const hg_opts* o) {
    hg_opts r;
    hg_opts_default(&r);
    if (o) r = *o;
    if (r.formulation != HG_FORM_FACE && r.formulation != HG_FORM_EDGE)
        throw Error{HG_E_INVALID_ARG, "formulation must be HG_FORM_FACE or HG_FORM_EDGE"};
    if (!(r.mu >= 0.0) || !std::isfinite(r.mu)) throw Error{HG_E_INVALID_ARG, "mu must be >= 0 (0 = auto)"};
    if (!(r.relax > 0.0 && r.relax < 2.0)) throw Error{HG_E_INVALID_ARG, "relax must lie in (0, 2)"};
    if (r.source_paths != 0 && r.source_paths != 1) throw Error{HG_E_INVALID_ARG, "source_paths must be 0 or 1"};
    if (r.cycle_constraints != 0 && r.cycle_constraints != 1)
        throw Error{HG_E_INVALID_ARG, "cycle_constraints must be 0 or 1"};
    if (r.use_graphs != 0 && r.use_graphs != 1) throw Error{HG_E_INVALID_ARG, "use_graphs must be 0 or 1"};
    if (r.t_per_component != 0 && r.t_per_component != 1)
        throw Error{HG_E_INVALID_ARG, "t_per_component must be 0 or 1"};
    if (!(r.tol_seam >= 0.0) || !std::isfinite(r.tol_seam)) throw Error{HG_E_INVALID_ARG, "tol_seam must be >= 0"};
    if (r.admm_block < 0 || r.admm_block > kMaxAdmmBlock)
        throw Error{HG_E_INVALID_ARG, "admm_block must lie in 0..8 (0 = auto)"};
    if (r.overlap_rings < 0 || r.overlap_rings > 4) throw Error{HG_E_INVALID_ARG, "overlap_rings must lie in 0..4"};
    if (r.diffusion_schedule < 0 || r.diffusion_schedule > 3)
        throw Error{HG_E_INVALID_ARG, "diffusion_schedule must lie in 0..3"};
    if (r.max_sweeps <= 0 || r.max_admm <= 0 || r.check_every <= 0)
        throw Error{HG_E_INVALID_ARG, "iteration caps must be positive"};
    return r;
}

// Diffusion time of each connected component: the given t > 0, else
// m hbar^2 (Eq. 27) with hbar the mean edge length of the whole mesh or,
// with opts.t_per_component, of the component itself.
static std::vector<double> resolve_t(const Mesh& m, double t, const hg_opts& o) {
    std::vector<double> tc(std::max(1, m.n_comp));
    const double mm = (o.m > 0.0 && std::isfinite(o.m)) ? o.m : 1.0;
    for (size_t c = 0; c < tc.size(); ++c) {
        double h = m.hbar;
        if (o.t_per_component && c < m.comp_hbar_host.size() && m.comp_hbar_host[c] > 0.0) h = m.comp_hbar_host[c];
        tc[c] = (t > 0.0 && std::isfinite(t)) ? t : mm * h * h;
    }
    return tc;
}


struct StageTimer {
    hipStream_t s;
    hipEvent_t ev[8];
    int n = 0;
    explicit StageTimer(hipStream_t st) : s(st) {
        for (auto& e : ev) HG_CHECK_HIP(hipEventCreate(&e));
    }
    ~StageTimer() {
        for (auto& e : ev) (void)hipEventDestroy(e);
    }
    void mark() { HG_CHECK_HIP(hipEventRecord(ev[n++], s)); }
    float ms(int a, int b) {
        float r = 0.f;
        HG_CHECK_HIP(hipEventSynchronize(ev[b]));
        HG_CHECK_HIP(hipEventElapsedTime(&r, ev[a], ev[b]));
        return r;
    }
};

}  // namespace hg

using namespace hg;

// One whole query (Algorithm 1) on workspace w and stream s.  Throws Error
// for invalid arguments and device failures; non-convergence is returned.
QueryOutcome hg::solve_query(Mesh& mesh_ref, Work& w, const int32_t* src, int32_t nsrc, double t, const hg_opts* opts,
                         float* d_dev, hipStream_t s, hg_info* info) {
    Mesh* m = &mesh_ref;
    w.ensure_pinned();
    hg_opts o = resolve_opts(opts);
    if (!s && o.use_graphs) {
        // the null stream cannot be captured: run on the workspace's own
        // stream, after what the caller queued on the null stream
        w.ensure_stream();
        HG_CHECK_HIP(hipEventRecord(w.ev, nullptr));
        HG_CHECK_HIP(hipStreamWaitEvent(w.own_stream, w.ev, 0));
        s = w.own_stream;
    }
    if (m->intrinsic && o.formulation == HG_FORM_FACE)
        throw Error{HG_E_INVALID_ARG, "the face form needs an extrinsic mesh (hg_mesh_create)"};
    auto si = map_sources(*m, src, nsrc);
    std::vector<double> tt = resolve_t(*m, t, o);
    StageTimer tm(s);
    tm.mark();
    const bool src_paths = nsrc > 1 && o.source_paths;
    const bool cycles = o.cycle_constraints && m->n_cycles > 0;
    const bool paths = src_paths || cycles;
    if (paths) build_constraint_paths(*m, w, si, src_paths, cycles, o.formulation, s);
    int depth = run_bfs(*m, w, si, s);
    tm.mark();
    DiffusionResult dr = run_diffusion(*m, w, si, tt, o, s);
    tm.mark();
    run_normalize(*m, w, s);
    tm.mark();
    // ADMM penalty: the low-frequency error of these iterations decays
    // fastest for mu of the order of the longest chain the field is
    // integrated along (measured, one source: best mu ~ 100 at depth 167,
    // ~ 300 at depth 663; several sources with path constraints: the
    // longest path's edge count, 20-32% fewer iterations than 1.5 times it
    // from 8 sources at level 6 to 32 at level 10; generator loops on a
    // torus: best mu ~ half the longest loop's edge count); mu = 0 picks
    // max(30, depth / 2, longest source path, longest loop / 2)
    if (o.mu == 0.0) {
        o.mu = std::max(30.0, 0.5 * depth);
        if (paths && w.paths.np > 0)
            o.mu = std::max({o.mu, 1.0 * w.paths.max_len_src, 0.5 * w.paths.max_len_cyc});
    }
    AdmmResult ar = o.formulation == HG_FORM_EDGE ? run_admm_edge(*m, w, 0, o, s, depth, paths)
                                                  : run_admm_face(*m, w, 0, o, s, depth, paths);
    tm.mark();
    integrate(*m, w, o.formulation, depth, d_dev, s);
    tm.mark();
    HG_CHECK_HIP(hipStreamSynchronize(s));
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->bfs_depth = depth;
        info->sweeps = dr.sweeps;
        info->passes = dr.passes;
        info->admm_iters = ar.iters;
        info->res_u = dr.res;
        info->res_primal = ar.rp;
        info->res_dual = ar.rd;
        info->t = tt[0];
        info->ms_bfs = tm.ms(0, 1);
        info->ms_diffusion = tm.ms(1, 2);
        info->ms_normalize = tm.ms(2, 3);
        info->ms_admm = tm.ms(3, 4);
        info->ms_integrate = tm.ms(4, 5);
        info->ms_total = tm.ms(0, 5);
        info->workspace_bytes = w.bytes();
        info->converged_u = dr.converged;
        info->converged_admm = ar.converged;
        info->ms_pass_kernel = dr.timed_launches ? (float)(dr.kernel_ms / dr.timed_launches) : 0.f;
        info->ms_admm_kernel = ar.timed_launches ? (float)(ar.kernel_ms / ar.timed_launches) : 0.f;
        info->bytes_pass_kernel = dr.bytes_per_pass;
        info->bytes_admm_kernel = ar.bytes_per_iter;
        info->bytes_alg = dr.bytes_per_pass * (uint64_t)dr.passes + ar.bytes_per_iter * (uint64_t)ar.launches;
        info->admm_launches = ar.launches;
        info->admm_block = ar.block;
        info->n_paths = paths ? w.paths.np_src : 0;
        info->path_edges = paths ? w.paths.ns_src : 0;
        info->n_cycles = paths ? w.paths.n_cyc : 0;
        info->cycle_slots = paths ? w.paths.ns_cyc : 0;
        info->seam = (float)ar.seam;
    }
    if (!dr.converged) return {HG_E_NOT_CONVERGED, "diffusion sweep cap reached"};
    if (!ar.converged) return {HG_E_NOT_CONVERGED, "ADMM iteration cap reached"};
    return {HG_OK, ""};
}

extern "C" {

hg_status hg_opts_default(hg_opts* o) {
    if (!o) return HG_E_INVALID_ARG;
    std::memset(o, 0, sizeof(*o));
    o->formulation = HG_FORM_EDGE;
    o->m = 1.0;
    o->tol_u = 1e-11;
    o->tol_admm = 1e-5;
    o->max_sweeps = 100000;
    o->max_admm = 50000;
    o->mu = 0.0;
    o->relax = 1.9;
    o->check_every = 32;
    o->diffusion_schedule = 0;
    o->inner_sweeps = 0;
    o->source_paths = 1;
    o->cycle_constraints = 1;
    o->use_graphs = 1;
    return HG_OK;
}

const char* hg_last_error(void) { return g_last_error.c_str(); }

// Mesh creation: from the caller's triangles, or (intrinsic) from the
// intrinsic Delaunay triangulation of them with the geometry taken from the
// intrinsic edge lengths.
// Tile workgroups that run at a time on the current device: the diffusion
// and breadth-first tile kernels fit two 1024-thread workgroups per CU.  0
// when there is no device to ask (the mesh is then refused later anyway).
static int tile_slots() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return 2 * cus;
}

static hg_status create_mesh(const double* xyz, int64_t nv, const int32_t* tri, int64_t nf, void* stream,
                             hg_mesh_t* out, bool intrinsic) {
    return guarded([&]() -> hg_status {
        if (!xyz || !tri || !out) return fail(HG_E_INVALID_ARG, "null argument");
        *out = nullptr;
        hipStream_t s = (hipStream_t)stream;
        IntrinsicTri idt;
        if (intrinsic) build_intrinsic(xyz, nv, tri, nf, idt);
        HostTopo T;
        build_topology(xyz, nv, intrinsic ? idt.tri.data() : tri, nf, 1024, T, tile_slots());
        build_cycles(T);
        std::vector<double> elen, floc;
        std::vector<int32_t> tile_k0;   // uploaded asynchronously: lives until geometry_init has synchronised
        if (intrinsic) {
            // per internal edge length; per internal face its corners in its
            // own plane, (0,0), (l01,0), (x2,y2) by the law of cosines
            elen.resize(T.ne);
            for (int64_t e = 0; e < T.ne; ++e)
                elen[e] = idt.edge_length(T.perm_v[T.ev[2 * e]], T.perm_v[T.ev[2 * e + 1]]);
            floc.resize(3 * T.nf);
            for (int64_t f = 0; f < T.nf; ++f) {
                double l[3];
                for (int k = 0; k < 3; ++k) l[k] = elen[slot_edge(T.fslot[3 * f + k])];
                const double x2 = (l[0] * l[0] + l[2] * l[2] - l[1] * l[1]) / (2.0 * l[0]);
                const double y2 = std::sqrt(std::max(l[2] * l[2] - x2 * x2, 0.0));
                floc[3 * f] = l[0];
                floc[3 * f + 1] = x2;
                floc[3 * f + 2] = y2;
                if (!(y2 > 0.0)) throw Error{HG_E_BAD_MESH, "degenerate intrinsic triangle"};
            }
            // t = m hbar^2 from the input mesh's edges (per component too)
            std::vector<double> len(T.n_comp, 0.0);
            std::vector<int64_t> cnt(T.n_comp, 0);
            for (size_t i = 0; i < idt.input_a.size(); ++i) {
                const int c = T.comp[T.iperm_v[idt.input_a[i]]];
                len[c] += idt.input_len[i];
                cnt[c]++;
            }
            for (int c = 0; c < T.n_comp; ++c) T.comp_hbar[c] = cnt[c] ? len[c] / (double)cnt[c] : 0.0;
        }
        auto* m = new Mesh();
        try {
            HG_CHECK_HIP(hipGetDevice(&m->device));
            m->intrinsic = intrinsic;
            if (intrinsic) {
                m->n_flips = idt.n_flips;
                m->n_nondelaunay = idt.n_nondelaunay;
                m->hbar = idt.hbar_input;
                m->floc.upload(floc, s);
                m->idt_tri_host = idt.tri;
                m->idt_len_canon.resize(T.ne);
                for (int64_t e = 0; e < T.ne; ++e) m->idt_len_canon[T.perm_e[e]] = elen[e];
            }
            m->nv = T.nv;
            m->nf = T.nf;
            m->ne = T.ne;
            m->nbnd = T.nbnd;
            m->max_valence = T.max_valence;
            m->iperm_v_host = T.iperm_v;
            m->px.upload(T.px, s);
            m->py.upload(T.py, s);
            m->pz.upload(T.pz, s);
            m->perm_v.upload(T.perm_v, s);
            m->perm_f.upload(T.perm_f, s);
            m->perm_e.upload(T.perm_e, s);
            m->row_ptr.upload(T.row_ptr, s);
            m->col.upload(T.col, s);
            m->csr_edge.upload(T.csr_edge, s);
            m->tri.upload(T.tri, s);
            m->fslot.upload(T.fslot, s);
            m->fsign.upload(T.fsign, s);
            m->ev.upload(T.ev, s);
            m->ef.upload(T.ef, s);
            m->twin.upload(T.twin, s);
            m->h01.upload(T.h01, s);
            m->patch_size = T.patch_size;
            m->n_patches = (int)(T.halo_ptr.size() - 1);
            m->max_halo = T.max_halo;
            m->max_ell_width = T.max_ell_width;
            m->tile_ptr.upload(T.tile_ptr, s);
            tile_k0.resize(T.tile_ptr.size());
            for (size_t p = 0; p < tile_k0.size(); ++p) tile_k0[p] = T.row_ptr[T.tile_ptr[p]];
            m->tile_k0.upload(tile_k0, s);
            m->tile_adj_ptr.upload(T.tile_adj_ptr, s);
            m->tile_adj.upload(T.tile_adj, s);
            m->halo_ptr.upload(T.halo_ptr, s);
            m->halo_idx.upload(T.halo_idx, s);
            m->ell_ptr.upload(T.ell_ptr, s);
            m->lnb.upload(T.lnb, s);
            m->ell_width.upload(T.ell_width, s);
            m->color_ptr_host = T.color_ptr;
            m->n_comp = T.n_comp;
            m->comp_hbar_host = T.comp_hbar;
            m->comp_v.upload(T.comp, s);
            m->tile_comp.upload(T.tile_comp, s);
            m->tile_order.upload(T.tile_order, s);
            m->n_cycles = T.n_cycles;
            m->cyc_e_ptr.swap(T.cyc_e_ptr);
            m->cyc_e_edge.swap(T.cyc_e_edge);
            m->cyc_e_sign.swap(T.cyc_e_sign);
            m->cyc_e_face.swap(T.cyc_e_face);
            m->cyc_e_canon.swap(T.cyc_e_canon);
            m->cyc_f_caller.swap(T.cyc_f_caller);
            m->cyc_f_ptr.swap(T.cyc_f_ptr);
            m->cyc_f_face.swap(T.cyc_f_face);
            m->cyc_f_edge.swap(T.cyc_f_edge);
            m->cyc_f_vec.swap(T.cyc_f_vec);
            m->w.ensure_pinned();
            geometry_init(*m, s, intrinsic ? &elen : nullptr);
        } catch (...) {
            delete m;
            throw;
        }
        *out = reinterpret_cast<hg_mesh_t>(m);
        return HG_OK;
    });
}

hg_status hg_mesh_create(const double* xyz, int64_t nv, const int32_t* tri, int64_t nf, void* stream,
                         hg_mesh_t* out) {
    return create_mesh(xyz, nv, tri, nf, stream, out, false);
}

hg_status hg_mesh_create_intrinsic(const double* xyz, int64_t nv, const int32_t* tri, int64_t nf, void* stream,
                                   hg_mesh_t* out) {
    return create_mesh(xyz, nv, tri, nf, stream, out, true);
}

hg_status hg_mesh_intrinsic(hg_mesh_t mesh, int32_t* tri_out, double* length_out) {
    return guarded([&]() -> hg_status {
        if (!mesh || !tri_out || !length_out) return fail(HG_E_INVALID_ARG, "null argument");
        auto* m = reinterpret_cast<Mesh*>(mesh);
        if (!m->intrinsic) return fail(HG_E_INVALID_ARG, "mesh was not created with hg_mesh_create_intrinsic");
        std::copy(m->idt_tri_host.begin(), m->idt_tri_host.end(), tri_out);
        std::copy(m->idt_len_canon.begin(), m->idt_len_canon.end(), length_out);
        return HG_OK;
    });
}

void hg_mesh_destroy(hg_mesh_t mesh) {
    if (!mesh) return;
    forget_joins_with(reinterpret_cast<Mesh*>(mesh));
    delete reinterpret_cast<Mesh*>(mesh);
}

uint64_t hg_mesh_bytes(hg_mesh_t mesh) { return mesh ? reinterpret_cast<Mesh*>(mesh)->mesh_bytes() : 0; }

uint64_t hg_query_bytes(hg_mesh_t mesh, int32_t nsrc, const hg_opts* opts) {
    if (!mesh || nsrc <= 0) return 0;
    const int form = opts ? opts->formulation : HG_FORM_EDGE;
    if (form != HG_FORM_EDGE && form != HG_FORM_FACE) return 0;
    return work_estimate(*reinterpret_cast<Mesh*>(mesh), form, nsrc);
}

hg_status hg_mesh_get_stats(hg_mesh_t mesh, hg_mesh_stats* st) {
    return guarded([&]() -> hg_status {
        if (!mesh || !st) return fail(HG_E_INVALID_ARG, "null argument");
        auto* m = reinterpret_cast<Mesh*>(mesh);
        std::memset(st, 0, sizeof(*st));
        st->nv = m->nv;
        st->nf = m->nf;
        st->ne = m->ne;
        st->n_boundary_edges = m->nbnd;
        st->hbar = m->hbar;
        st->total_area = m->total_area;
        st->max_valence = m->max_valence;
        st->n_patches = m->n_patches;
        st->mesh_bytes = m->mesh_bytes();
        st->n_components = m->n_comp;
        st->n_colors = (int32_t)m->color_ptr_host.size() - 1;
        st->n_cycles = m->n_cycles;
        st->cycle_edges = (int32_t)m->cyc_e_edge.size();
        st->cycle_faces = (int32_t)m->cyc_f_face.size();
        st->intrinsic = m->intrinsic ? 1 : 0;
        st->n_flips = (int32_t)m->n_flips;
        st->n_nondelaunay = (int32_t)m->n_nondelaunay;
        return HG_OK;
    });
}

hg_status hg_mesh_cycles(hg_mesh_t mesh, int32_t form, int32_t* ptr, int32_t* ids, float* coef, int64_t capacity) {
    return guarded([&]() -> hg_status {
        if (!mesh || !ptr || !ids || !coef) return fail(HG_E_INVALID_ARG, "null argument");
        if (form != HG_FORM_EDGE && form != HG_FORM_FACE)
            return fail(HG_E_INVALID_ARG, "form must be HG_FORM_FACE or HG_FORM_EDGE");
        auto* m = reinterpret_cast<Mesh*>(mesh);
        const bool ef = form == HG_FORM_EDGE;
        const auto& p = ef ? m->cyc_e_ptr : m->cyc_f_ptr;
        const auto& id = ef ? m->cyc_e_canon : m->cyc_f_caller;
        const auto& cf = ef ? m->cyc_e_sign : m->cyc_f_vec;
        if (capacity < (int64_t)id.size()) return fail(HG_E_INVALID_ARG, "capacity below the loops' slot count");
        std::copy(p.begin(), p.end(), ptr);
        std::copy(id.begin(), id.end(), ids);
        std::copy(cf.begin(), cf.end(), coef);
        return HG_OK;
    });
}

hg_status hg_mesh_edges(hg_mesh_t mesh, int32_t* edges_dev, void* stream) {
    return guarded([&]() -> hg_status {
        if (!mesh || !edges_dev) return fail(HG_E_INVALID_ARG, "null argument");
        auto* m = reinterpret_cast<Mesh*>(mesh);
        hipStream_t s = (hipStream_t)stream;
        edges_to_user(*m, edges_dev, s);
        HG_CHECK_HIP(hipStreamSynchronize(s));
        return HG_OK;
    });
}

hg_status hg_mesh_weights(hg_mesh_t mesh, double* theta_dev, double* area_dev, void* stream) {
    return guarded([&]() -> hg_status {
        if (!mesh || (!theta_dev && !area_dev)) return fail(HG_E_INVALID_ARG, "null argument");
        auto* m = reinterpret_cast<Mesh*>(mesh);
        hipStream_t s = (hipStream_t)stream;
        weights_to_user(*m, theta_dev, area_dev, s);
        HG_CHECK_HIP(hipStreamSynchronize(s));
        return HG_OK;
    });
}

hg_status hg_bfs(hg_mesh_t mesh, const int32_t* src, int32_t nsrc, int32_t* level_dev, int32_t* parent_dev,
                 void* stream, int32_t* depth_out) {
    return guarded([&]() -> hg_status {
        if (!mesh) return fail(HG_E_INVALID_ARG, "null mesh");
        auto* m = reinterpret_cast<Mesh*>(mesh);
        hipStream_t s = (hipStream_t)stream;
        auto si = map_sources(*m, src, nsrc);
        int depth = run_bfs(*m, m->w, si, s);
        if (level_dev) scatter_vertices_to_user_i(*m, m->w.level.p, level_dev, false, s);
        if (parent_dev) scatter_vertices_to_user_i(*m, m->w.parent.p, parent_dev, true, s);
        HG_CHECK_HIP(hipStreamSynchronize(s));
        if (depth_out) *depth_out = depth;
        return HG_OK;
    });
}

hg_status hg_diffuse(hg_mesh_t mesh, const int32_t* src, int32_t nsrc, double t, const hg_opts* opts,
                     double* logu_dev, void* stream, hg_info* info) {
    return guarded([&]() -> hg_status {
        if (!mesh || !logu_dev) return fail(HG_E_INVALID_ARG, "null argument");
        auto* m = reinterpret_cast<Mesh*>(mesh);
        hipStream_t s = (hipStream_t)stream;
        hg_opts o = resolve_opts(opts);
        auto si = map_sources(*m, src, nsrc);
        std::vector<double> tt = resolve_t(*m, t, o);
        int depth = run_bfs(*m, m->w, si, s);
        DiffusionResult r = run_diffusion(*m, m->w, si, tt, o, s);
        diffusion_logu(*m, m->w, s);
        scatter_vertices_to_user_d(*m, m->w.logu.p, logu_dev, s);
        HG_CHECK_HIP(hipStreamSynchronize(s));
        if (info) {
            std::memset(info, 0, sizeof(*info));
            info->bfs_depth = depth;
            info->sweeps = r.sweeps;
            info->passes = r.passes;
            info->res_u = r.res;
            info->t = tt[0];
            info->converged_u = r.converged;
        }
        return r.converged ? HG_OK : fail(HG_E_NOT_CONVERGED, "diffusion sweep cap reached");
    });
}

hg_status hg_normalize(hg_mesh_t mesh, const double* logu_dev, float* h_dev, void* stream) {
    return guarded([&]() -> hg_status {
        if (!mesh || !logu_dev || !h_dev) return fail(HG_E_INVALID_ARG, "null argument");
        auto* m = reinterpret_cast<Mesh*>(mesh);
        hipStream_t s = (hipStream_t)stream;
        normalize_from_logu(*m, m->w, logu_dev, s);
        scatter_faces_to_user(*m, m->w.h.p, h_dev, s);
        HG_CHECK_HIP(hipStreamSynchronize(s));
        return HG_OK;
    });
}

static hg_status admm_stage(hg_mesh_t mesh, const float* h_dev, const int32_t* src, int32_t nsrc, int32_t iters,
                            const hg_opts* opts, float* out, void* stream, hg_info* info, int form) {
    return guarded([&]() -> hg_status {
        if (!mesh || !h_dev || !out) return fail(HG_E_INVALID_ARG, "null argument");
        auto* m = reinterpret_cast<Mesh*>(mesh);
        hipStream_t s = (hipStream_t)stream;
        hg_opts o = resolve_opts(opts);
        if (m->intrinsic && form == HG_FORM_FACE)
            return fail(HG_E_INVALID_ARG, "the face form needs an extrinsic mesh (hg_mesh_create)");
        if (o.mu == 0.0) o.mu = 100.0;   // no breadth-first depth here: the paper's value
        const bool src_paths = src && nsrc > 1 && o.source_paths;
        const bool cycles = o.cycle_constraints && m->n_cycles > 0;
        const bool paths = src_paths || cycles;
        if (paths)
            build_constraint_paths(*m, m->w, src_paths ? map_sources(*m, src, nsrc) : std::vector<int32_t>{},
                                   src_paths, cycles, form, s);
        m->w.h.alloc((size_t)3 * m->nf);
        gather_faces_to_internal(*m, h_dev, m->w.h.p, s);
        AdmmResult r = form == HG_FORM_EDGE ? run_admm_edge(*m, m->w, iters, o, s, -1, paths)
                                            : run_admm_face(*m, m->w, iters, o, s, -1, paths);
        if (form == HG_FORM_EDGE)
            scatter_edges_to_user(*m, m->w.xe.p, out, s);
        else
            scatter_faces_to_user(*m, m->w.gf.p, out, s);
        HG_CHECK_HIP(hipStreamSynchronize(s));
        if (info) {
            std::memset(info, 0, sizeof(*info));
            info->admm_iters = r.iters;
            info->res_primal = r.rp;
            info->res_dual = r.rd;
            info->converged_admm = r.converged;
            info->n_paths = paths ? m->w.paths.np_src : 0;
            info->path_edges = paths ? m->w.paths.ns_src : 0;
            info->n_cycles = paths ? m->w.paths.n_cyc : 0;
            info->cycle_slots = paths ? m->w.paths.ns_cyc : 0;
            info->admm_launches = r.launches;
            info->admm_block = r.block;
        }
        return r.converged ? HG_OK : fail(HG_E_NOT_CONVERGED, "ADMM iteration cap reached");
    });
}

hg_status hg_admm_edge(hg_mesh_t mesh, const float* h_dev, const int32_t* src, int32_t nsrc, int32_t iters,
                       const hg_opts* opts, float* x_dev, void* stream, hg_info* info) {
    return admm_stage(mesh, h_dev, src, nsrc, iters, opts, x_dev, stream, info, HG_FORM_EDGE);
}

hg_status hg_admm_face(hg_mesh_t mesh, const float* h_dev, const int32_t* src, int32_t nsrc, int32_t iters,
                       const hg_opts* opts, float* g_dev, void* stream, hg_info* info) {
    return admm_stage(mesh, h_dev, src, nsrc, iters, opts, g_dev, stream, info, HG_FORM_FACE);
}

static hg_status integrate_stage(hg_mesh_t mesh, const int32_t* src, int32_t nsrc, const float* in, float* d_dev,
                                 void* stream, int form) {
    return guarded([&]() -> hg_status {
        if (!mesh || !in || !d_dev) return fail(HG_E_INVALID_ARG, "null argument");
        auto* m = reinterpret_cast<Mesh*>(mesh);
        hipStream_t s = (hipStream_t)stream;
        if (m->intrinsic && form == HG_FORM_FACE)
            return fail(HG_E_INVALID_ARG, "the face form needs an extrinsic mesh (hg_mesh_create)");
        auto si = map_sources(*m, src, nsrc);
        int depth = run_bfs(*m, m->w, si, s);
        if (form == HG_FORM_EDGE) {
            m->w.xe.alloc(m->ne);
            gather_edges_to_internal(*m, in, m->w.xe.p, s);
        } else {
            m->w.gf.alloc((size_t)3 * m->nf);
            gather_faces_to_internal(*m, in, m->w.gf.p, s);
        }
        integrate(*m, m->w, form, depth, d_dev, s);
        HG_CHECK_HIP(hipStreamSynchronize(s));
        return HG_OK;
    });
}

hg_status hg_integrate_edge(hg_mesh_t mesh, const int32_t* src, int32_t nsrc, const float* x_dev, float* d_dev,
                            void* stream) {
    return integrate_stage(mesh, src, nsrc, x_dev, d_dev, stream, HG_FORM_EDGE);
}

hg_status hg_integrate_face(hg_mesh_t mesh, const int32_t* src, int32_t nsrc, const float* g_dev, float* d_dev,
                            void* stream) {
    return integrate_stage(mesh, src, nsrc, g_dev, d_dev, stream, HG_FORM_FACE);
}

hg_status hg_mesh_autotune(hg_mesh_t mesh, const int32_t* src, int32_t nsrc, double t, const hg_opts* opts,
                           void* stream, hg_tune_report* report) {
    return guarded([&]() -> hg_status {
        if (!mesh) return fail(HG_E_INVALID_ARG, "null argument");
        auto* m = reinterpret_cast<Mesh*>(mesh);
        hipStream_t s = (hipStream_t)stream;
        hg_opts o = resolve_opts(opts);
        auto si = map_sources(*m, src, nsrc);
        std::vector<double> tt = resolve_t(*m, t, o);
        Work& w = m->w;
        w.ensure_pinned();
        run_bfs(*m, w, si, s);
        struct Cand {
            int sched, inner, rings;
        };
        // global Jacobi needs more sweeps than the breadth-first depth: it is a
        // candidate only on meshes of a few tiles (or without tiles)
        std::vector<Cand> cands;
        if (!patch_supported(*m) || m->n_patches <= 16) cands.push_back({1, 0, 0});
        if (patch_supported(*m)) {
            for (int inner : {16, 32, 64}) cands.push_back({2, inner, 0});
            const int r0 = o.overlap_rings > 0 ? o.overlap_rings : 1;
            for (int rings : {r0, r0 + 1})
                if (rings <= 4)
                    for (int inner : {32, 64}) cands.push_back({3, inner, rings});
        }
        hg_tune_report rep;
        std::memset(&rep, 0, sizeof(rep));
        rep.n_candidates = (int)cands.size();
        rep.chosen = -1;
        rep.admm_chosen = -1;
        hipEvent_t a, b;
        HG_CHECK_HIP(hipEventCreate(&a));
        HG_CHECK_HIP(hipEventCreate(&b));
        float best = 0.f;
        const int saved_sched = m->tuned_schedule, saved_inner = m->tuned_inner, saved_rings = m->tuned_rings;
        size_t overlap_sets_before;
        {
            std::lock_guard<std::mutex> lock(m->ot_mu);
            overlap_sets_before = m->otiles.size();
        }
        try {
            m->tuned_schedule = m->tuned_inner = m->tuned_rings = 0;
            for (size_t i = 0; i < cands.size(); ++i) {
                hg_opts oc = o;
                oc.diffusion_schedule = cands[i].sched;
                oc.inner_sweeps = cands[i].inner;
                oc.overlap_rings = cands[i].rings;
                HG_CHECK_HIP(hipEventRecord(a, s));
                DiffusionResult dr;
                try {
                    dr = run_diffusion(*m, w, si, tt, oc, s);
                } catch (const Error& e) {
                    // overlapping tiles that do not fit this mesh: not a candidate
                    if (e.code != HG_E_INVALID_ARG || cands[i].sched != 3) throw;
                    dr = DiffusionResult();
                }
                HG_CHECK_HIP(hipEventRecord(b, s));
                HG_CHECK_HIP(hipEventSynchronize(b));
                float ms = 0.f;
                HG_CHECK_HIP(hipEventElapsedTime(&ms, a, b));
                rep.schedule[i] = cands[i].sched;
                rep.inner_sweeps[i] = cands[i].inner;
                rep.overlap_rings[i] = cands[i].rings;
                rep.ms[i] = ms;
                rep.passes[i] = dr.passes;
                if (dr.converged && (rep.chosen < 0 || ms < best)) {
                    best = ms;
                    rep.chosen = (int)i;
                }
            }
        } catch (...) {
            m->tuned_schedule = saved_sched;
            m->tuned_inner = saved_inner;
            m->tuned_rings = saved_rings;
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            throw;
        }
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        if (rep.chosen >= 0) {
            m->tuned_schedule = cands[rep.chosen].sched;
            m->tuned_inner = cands[rep.chosen].inner;
            m->tuned_rings = cands[rep.chosen].rings;
        } else {
            m->tuned_schedule = saved_sched;
            m->tuned_inner = saved_inner;
            m->tuned_rings = saved_rings;
        }
        // overlapping tiles built only for this trial are not kept unless chosen
        {
            HG_CHECK_HIP(hipStreamSynchronize(s));
            std::lock_guard<std::mutex> lock(m->ot_mu);
            auto& ot = m->otiles;
            for (size_t i = ot.size(); i-- > overlap_sets_before;)
                if (m->tuned_schedule != 3 || ot[i]->rings != m->tuned_rings) ot.erase(ot.begin() + i);
        }
        // the edge form's ADMM block: the same iterations (their count a
        // multiple of every candidate) timed for each, from the probe's
        // normalised field; face tiles built for the trial are kept only
        // for the block chosen
        if (rep.chosen >= 0 && o.formulation == HG_FORM_EDGE && o.admm_block == 0) {
            run_diffusion(*m, w, si, tt, o, s);
            run_normalize(*m, w, s);
            hg_opts oa = o;
            if (oa.mu == 0.0) oa.mu = 100.0;   // timing only: the arithmetic per iteration does not depend on mu
            oa.check_every = 64;               // runs of 64 iterations, as a solve's between two checks
            size_t edge_sets_before;
            {
                std::lock_guard<std::mutex> lock(m->et_mu);
                edge_sets_before = m->etiles.size();
            }
            const int saved_block = m->tuned_admm_block;
            float best_us = 0.f;
            int nb = 0;
            for (int kb : {4, 5, 6}) {
                oa.admm_block = kb;
                AdmmResult r0 = run_admm_edge(*m, w, 64, oa, s);   // builds the face tiles, warms up
                if (r0.block != kb) continue;                          // regions of kb rings do not fit
                HG_CHECK_HIP(hipEventCreate(&a));
                HG_CHECK_HIP(hipEventCreate(&b));
                HG_CHECK_HIP(hipEventRecord(a, s));
                run_admm_edge(*m, w, 192, oa, s);
                HG_CHECK_HIP(hipEventRecord(b, s));
                HG_CHECK_HIP(hipEventSynchronize(b));
                float ms = 0.f;
                HG_CHECK_HIP(hipEventElapsedTime(&ms, a, b));
                (void)hipEventDestroy(a);
                (void)hipEventDestroy(b);
                rep.admm_block[nb] = kb;
                rep.admm_us_per_iteration[nb] = 1e3f * ms / 192.f;
                if (rep.admm_chosen < 0 || rep.admm_us_per_iteration[nb] < best_us) {
                    best_us = rep.admm_us_per_iteration[nb];
                    rep.admm_chosen = nb;
                }
                ++nb;
            }
            rep.n_admm = nb;
            m->tuned_admm_block = rep.admm_chosen >= 0 ? rep.admm_block[rep.admm_chosen] : saved_block;
            HG_CHECK_HIP(hipStreamSynchronize(s));
            std::lock_guard<std::mutex> lock(m->et_mu);
            auto& et = m->etiles;
            for (size_t i = et.size(); i-- > edge_sets_before;)
                if (et[i]->rings != m->tuned_admm_block) et.erase(et.begin() + i);
        }
        if (report) *report = rep;
        return rep.chosen >= 0 ? HG_OK : fail(HG_E_NOT_CONVERGED, "no candidate schedule converged");
    });
}

hg_status hg_geodesic_solve(hg_mesh_t mesh, const int32_t* src, int32_t nsrc, double t, const hg_opts* opts,
                            float* d_dev, void* stream, hg_info* info) {
    return guarded([&]() -> hg_status {
        if (!mesh || !d_dev) return fail(HG_E_INVALID_ARG, "null argument");
        auto* m = reinterpret_cast<Mesh*>(mesh);
        QueryOutcome q = solve_query(*m, m->w, src, nsrc, t, opts, d_dev, (hipStream_t)stream, info);
        return q.status == HG_OK ? HG_OK : fail(q.status, q.msg);
    });
}

}  // extern "C"
