/*
 * hgeo -- the parallel heat method for geodesic distance on triangle meshes
 * (Tao, Zhang, Deng, Fang, Peng, He: "Parallel and Scalable Heat Methods for
 * Geodesic Distance Computation", arXiv 1812.06060), as a C ABI over HIP
 * kernels for AMD Instinct MI355X (gfx950).
 *
 * Pipeline of one solve (Algorithm 1 of the paper):
 *   1. breadth-first vertex sets D_i from the sources and the pairing of each
 *      vertex with a neighbour one set closer (Eq. 6, Sec. 3.3);
 *   2. heat diffusion (A - t L_c) u = u_0 (Eq. 4) by sweep iterations of the
 *      update Eq. 7, in FP64 with a per-vertex binary exponent so that u
 *      never underflows;
 *   3. face-wise normalisation h = -grad u / |grad u| (Eq. 3), plus the edge
 *      targets of Eq. 18 for the edge form;
 *   4. ADMM optimisation of integrable gradients: face form (Sec. 3.2,
 *      Eqs. 9-16) or edge form (Sec. 4.1, Eqs. 19-21), FP32;
 *   5. integration of the optimised gradients along the pairing (Eq. 17 and
 *      Sec. 4), FP32 with compensated (double-float) summation.
 *
 * Conventions shared by every entry point:
 *   - Vertex, face and edge arrays passed in or out are in the caller's
 *     order: vertices and faces as given to hg_mesh_create, edges in the
 *     canonical order = unique undirected edges sorted by (min id, max id).
 *     The orientation halfedge of an edge runs from its smaller to its larger
 *     vertex id; an edge difference is x_e = d(larger) - d(smaller).
 *   - Source lists are HOST int32 arrays of vertex ids (duplicates ignored).
 *   - Every other array argument named *_dev is a DEVICE pointer on the
 *     current HIP device, caller-owned; the library only reads or writes it.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued
 *     on it; an entry point returns after its results are written (it waits
 *     on the stream to read convergence flags).
 *   - Errors are reported by status code; hg_last_error() returns a
 *     thread-local message for the last failing call.  No C++ exception
 *     crosses the ABI.  A failed call leaves existing meshes usable.
 */
#ifndef HGEO_H
#define HGEO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hg_mesh_s* hg_mesh_t;

typedef enum {
    HG_OK = 0,
    HG_E_INVALID_ARG = 1,   /* null pointer, bad size, source out of range, ... */
    HG_E_BAD_MESH = 2,      /* index out of range, degenerate face, non-manifold
                               edge, inconsistent orientation */
    HG_E_OOM = 3,           /* device allocation failed */
    HG_E_NOT_CONVERGED = 4, /* iteration cap reached; results are still written */
    HG_E_DEVICE = 5         /* a HIP call failed */
} hg_status;

enum { HG_FORM_FACE = 0, HG_FORM_EDGE = 1 };

/* Solve options.  hg_opts_default() fills the defaults listed here. */
typedef struct {
    int32_t formulation;    /* HG_FORM_EDGE (default) or HG_FORM_FACE */
    double m;               /* t = m * hbar^2 when the solve's t <= 0
                               (Eq. 27, hbar = mean edge length); default 1 */
    double tol_u;           /* diffusion: stop when the largest relative change
                               of u over one sweep is <= tol_u; default 1e-11 */
    double tol_admm;        /* ADMM stopping tolerance, default 1e-5.  In
                               hg_geodesic_solve: stop when the estimated
                               remaining change of the integrated distance
                               field is <= tol_admm * max d.  In the ADMM step
                               entry points: stop when the primal and dual
                               residuals are <= tol_admm (scales below). */
    int32_t max_sweeps;     /* diffusion sweep cap; default 100000 */
    int32_t max_admm;       /* ADMM iteration cap; default 50000 */
    double mu;              /* ADMM penalty (the paper uses 100); default 0 =
                               auto: max(30, depth/2, L, C/2) in
                               hg_geodesic_solve (depth = breadth-first depth
                               of the query, L = edges on the longest source
                               path, C = edges on the longest generator loop
                               of the cycle constraints, 0 without them), 100
                               in the ADMM step entry points */
    int32_t check_every;    /* iterations between convergence checks; 32 */
    int32_t diffusion_schedule; /* 0 = auto, 1 = global Jacobi sweeps,
                                   2 = LDS-tiled patch sweeps, 3 = LDS
                                   tiles that also sweep overlap_rings
                                   rings of vertices around their own (an
                                   overlapping Schwarz iteration: the same
                                   fixed point in fewer passes) */
    int32_t inner_sweeps;   /* patch schedule: sweeps per global pass; 0 = auto */
    double relax;           /* ADMM over-relaxation alpha in (0, 2); default
                               1.9 (measured: 4-21% fewer edge-form
                               iterations than 1.8 on the test workloads);
                               1 = the paper's iteration */
    int32_t source_paths;   /* several sources: 1 (default) adds the
                               constraints of Eqs. 24-25 (Sec. 5.2) along a
                               shortest edge path from the first source of
                               each connected component to each other source
                               in it, so that the optimised field gives every
                               source the same distance; 0 = without them */
    int32_t t_per_component; /* 1: when t <= 0, each connected component
                               uses t = m hbar_c^2 with hbar_c its own mean
                               edge length, so a mesh made of several
                               meshes side by side (a batch in one solve)
                               gives each the result it has alone;
                               0 (default): hbar of the whole mesh */
    int32_t use_graphs;     /* 1 (default): the launches between two
                               convergence checks are captured once into a
                               HIP graph and replayed; on the null stream the
                               solve runs on a stream of its own, ordered
                               after the caller's work on the null stream;
                               0: plain launches */
    int32_t cycle_constraints; /* 1 (default): on a closed component of
                               genus g > 0 the ADMM also constrains the
                               field's circulation around 2g generator
                               loops to zero (Sec. 5.1, Eq. 23 edge form,
                               Eq. 22 face form), so that it is the gradient
                               of a function there; 0 = without them.
                               Components with boundary get none. */
    double tol_seam;        /* hg_geodesic_solve: once the distance check is
                               met, also measure the seam, max over edges of
                               |d_head - d_tail - x_e| / hbar (d the field
                               integrated along the breadth-first tree, x_e
                               the edge difference of the optimised field;
                               zero on the tree's edges, elsewhere the jump
                               left by what is still not a gradient), and
                               stop only once it is <= tol_seam as well
                               (otherwise measure it again at every later
                               check);
                               default 0 = not required (it is reported in
                               hg_info.seam either way) */
    int32_t admm_block;     /* edge form without constraint groups: ADMM
                               iterations per launch, 1..8.  k > 1 runs k
                               iterations over face tiles held in LDS with a
                               halo of k rings of faces, with the result of k
                               single-iteration launches (the same
                               arithmetic) for fewer HBM bytes per
                               iteration.  A mesh whose regions do not fit
                               (at most 4096 faces each) uses the largest
                               smaller k that fits; every solve with source
                               paths or generator loops, and the face form,
                               run one iteration per launch
                               (hg_info.admm_block reports what was used).
                               Between two checks the iterations run in
                               launches of k and one launch of the rest, so
                               the result, the iteration count included, is
                               the same for every k.  0 = auto (default: the
                               block hg_mesh_autotune chose for the mesh,
                               else 6) */
    int32_t overlap_rings;  /* schedule 3: rings of overlap around each tile,
                               1..4 (a tile whose region would not fit the
                               LDS gets fewer); 0 = auto: the autotuned
                               count, else 2 */
} hg_opts;

/* Per-solve report. */
typedef struct {
    int32_t bfs_depth;      /* largest breadth-first level reached */
    int32_t sweeps;         /* diffusion sweeps performed (all schedules) */
    int32_t passes;         /* diffusion global passes (= sweeps for Jacobi) */
    int32_t admm_iters;     /* ADMM iterations performed */
    double res_u;           /* final largest relative sweep change of u */
    double res_primal;      /* final ADMM primal residual (form's scale) */
    double res_dual;        /* final ADMM dual residual (form's scale) */
    double t;               /* diffusion time used (of component 0 when
                               t_per_component is set) */
    float ms_bfs, ms_diffusion, ms_normalize, ms_admm, ms_integrate, ms_total;
    uint64_t bytes_alg;     /* algorithmic HBM bytes of the solve's kernels */
    uint64_t workspace_bytes; /* device bytes held for this mesh's queries */
    int32_t converged_u, converged_admm;
    /* average device time of one diffusion pass and of one launch of the
       main ADMM kernel (up to admm_block iterations: see admm_launches),
       from HIP events around back-to-back launches on the solve's stream,
       and the algorithmic HBM bytes one such launch moves */
    float ms_pass_kernel, ms_admm_kernel;
    uint64_t bytes_pass_kernel, bytes_admm_kernel;
    int32_t n_paths;        /* source paths constrained (Eqs. 24-25) */
    int32_t path_edges;     /* total edges over those paths */
    int32_t n_cycles;       /* generator loops constrained (Sec. 5.1) */
    int32_t cycle_slots;    /* total edges (edge form) or faces (face form)
                               over those loops */
    float seam;             /* hg_geodesic_solve: the last check's largest
                               seam / hbar (see hg_opts.tol_seam) */
    int32_t admm_launches;  /* launches of the main ADMM kernel: between
                               two checks, launches of admm_block
                               iterations and one of the rest
                               (ms_admm_kernel and bytes_admm_kernel are
                               per launch; admm_iters / admm_launches
                               iterations per launch on average) */
    int32_t admm_block;     /* iterations per launch actually used (1: one
                               iteration per launch) */
    int32_t reserved[1];
} hg_info;

/* Mesh statistics. */
typedef struct {
    int64_t nv, nf, ne, n_boundary_edges;
    double hbar;            /* mean edge length (Eq. 27) */
    double total_area;
    int32_t max_valence;
    int32_t n_patches;      /* LDS tiles of the patch diffusion schedule */
    uint64_t mesh_bytes;    /* device bytes held by the mesh */
    int32_t n_components;   /* connected components (vertex adjacency) */
    int32_t n_colors;       /* colours of the diffusion tiles */
    int32_t n_cycles;       /* generator loops: 2g per closed component of
                               genus g (Sec. 5.1), 0 for a component with
                               boundary */
    int32_t cycle_edges;    /* edges over the edge loops */
    int32_t cycle_faces;    /* faces over the face loops */
    int32_t intrinsic;      /* 1: built by hg_mesh_create_intrinsic */
    int32_t n_flips;        /* edge flips of the intrinsic Delaunay build */
    int32_t n_nondelaunay;  /* interior edges left non-Delaunay (flip would
                               have duplicated an edge) */
    int32_t reserved[4];
} hg_mesh_stats;

/* Fill *opts with the defaults above. */
hg_status hg_opts_default(hg_opts* opts);

/*
 * Build a resident device mesh (Sec. 3: manifold triangle mesh M=(V,E,F)).
 *   xyz  : HOST float64[nv*3] vertex positions.
 *   tri  : HOST int32[nf*3] counter-clockwise triangles (0-based ids).
 * Validates indices, rejects degenerate faces, edges with more than two
 * faces and inconsistently oriented neighbours (HG_E_BAD_MESH).  Computes on
 * the GPU: face areas, cotangent weights theta_jk = (cot a + cot b)/2, lumped
 * vertex areas A_j = (1/3) sum of incident face areas (Sec. 3.1), the mean
 * edge length; builds the breadth-first/LDS-tile schedules' connectivity.
 * The connectivity, tiles and colours are built on host worker threads: the
 * environment variable HG_HOST_THREADS sets their number (read once per
 * process; default the hardware's, at most 16); every table is the same for
 * any number of them.
 * The mesh owns its device memory until hg_mesh_destroy.
 */
hg_status hg_mesh_create(const double* xyz, int64_t nv, const int32_t* tri, int64_t nf,
                         void* stream, hg_mesh_t* out);

/*
 * The same on the intrinsic Delaunay triangulation of the mesh (Sec. 5.3):
 * the surface is described by connectivity and edge lengths, and interior
 * edges whose two facing angles sum beyond pi are flipped (first-in-first-
 * out queue over interior edges, initially in canonical order; the new
 * length from unfolding the two triangles into the plane; a flip that would
 * join two already joined vertices is skipped and the edge counted in
 * n_nondelaunay).  Breadth-first sets use the flipped connectivity; areas
 * and cotangent weights come from the intrinsic lengths; gradients and edge
 * targets (Eqs. 3, 18) are taken in each face's own frame (first vertex at
 * the origin, first edge along +x, third vertex at y > 0); t = m hbar^2
 * uses the mean edge length of the input mesh.  Only the edge form runs on
 * such a mesh (HG_E_INVALID_ARG for the face form).  Faces and edges seen
 * by the caller (face-indexed and edge-indexed arrays, hg_mesh_edges) are
 * those of the flipped triangulation: face i is row i of the flipped
 * triangle list.  The flips run on the host (time roughly linear in the
 * mesh size).
 */
hg_status hg_mesh_create_intrinsic(const double* xyz, int64_t nv, const int32_t* tri, int64_t nf,
                                   void* stream, hg_mesh_t* out);
/* The intrinsic triangulation of such a mesh: tri_out = HOST int32[nf*3]
 * flipped triangles (caller vertex ids), length_out = HOST float64[ne]
 * edge lengths in canonical edge order.  HG_E_INVALID_ARG for a mesh built
 * by hg_mesh_create. */
hg_status hg_mesh_intrinsic(hg_mesh_t mesh, int32_t* tri_out, double* length_out);

void hg_mesh_destroy(hg_mesh_t mesh);
hg_status hg_mesh_get_stats(hg_mesh_t mesh, hg_mesh_stats* stats);

/*
 * Geodesic distance from a source set (Algorithm 1; several sources as in
 * Sec. 5.2: all in D_0, u_0 = 1 at each, distance 0 at each, and with
 * opts->source_paths the path constraints of Eqs. 24-25 in the ADMM; the
 * paths come from a breadth-first search grown from the first source of
 * each component alone, which adds one search of that depth to the query).
 *   src, nsrc : HOST int32 source vertex ids, nsrc >= 1.
 *   t         : diffusion time; t <= 0 means m * hbar^2.
 *   opts      : NULL = defaults.
 *   d_dev     : DEVICE float32[nv] output distances (caller order);
 *               vertices not connected to a source get +inf.
 *   info      : optional report.
 * ADMM stops on the distance field: every check_every (>= 64) iterations the
 * current gradients are integrated; with delta the largest change of d since
 * the previous check and r the ratio of the last two changes, it stops when
 * delta r / (1 - r) <= tol_admm max d.  info reports the paper's residuals
 * at the end: face form |r_p|/|M|_F and |r_d|/|M|_F (Sec. 3.2); edge form
 * rms(r_p)/hbar and rms(r_d)/(mu hbar) over the 3|F| copies.
 * Returns HG_E_NOT_CONVERGED (results written) if a cap was hit.
 */
hg_status hg_geodesic_solve(hg_mesh_t mesh, const int32_t* src, int32_t nsrc, double t,
                            const hg_opts* opts, float* d_dev, void* stream, hg_info* info);

/*
 * Queries on several resident meshes in one solve (Algorithm 1 once for all
 * of them; a source list per mesh as in Sec. 5.2): query i runs on meshes[i]
 * from the HOST int32 source ids src[i][0 .. nsrc[i]) (its own vertex ids)
 * and writes DEVICE float32[nv of meshes[i]] d_dev[i].  The meshes are joined
 * on the device as the connected components of one mesh (their arrays
 * concatenated with shifted indices; nothing is rebuilt on the host), so
 * every step of the path runs one launch sequence for the whole batch.  Each
 * member diffuses with its own t = m hbar_i^2 when t <= 0 (t > 0 applies to
 * all), its breadth-first sets, tiles and source paths stay inside it, and
 * it gets the distance it has alone, to the solve's tolerances (the ADMM
 * stopping rule and the automatic penalty see the whole batch).  opts as in
 * hg_geodesic_solve (t_per_component is set by the call); info reports the
 * batch solve.  The join is kept for the next batch over the same meshes in
 * the same order (it holds a copy of their device arrays plus a workspace,
 * about as much as the members' own), and is freed when a batch over other
 * meshes is run or one of its members is destroyed.  A mesh may appear more
 * than once.  All meshes must live on the current device and be all
 * extrinsic or all intrinsic (HG_E_INVALID_ARG).  Batch calls are serialised
 * by the library.  Returns HG_E_NOT_CONVERGED (results written) if a cap was
 * hit.
 */
hg_status hg_geodesic_solve_batch(const hg_mesh_t* meshes, int32_t nq, const int32_t* const* src,
                                  const int32_t* nsrc, double t, const hg_opts* opts, float* const* d_dev,
                                  void* stream, hg_info* info);

/* Device bytes held by a mesh (its arrays and the schedules built so far);
 * 0 for NULL. */
uint64_t hg_mesh_bytes(hg_mesh_t mesh);
/* Upper estimate of the device bytes of one query's workspace on this mesh
 * with nsrc sources in the form of opts (NULL: edge form): breadth-first
 * sets, diffusion state, normalised field, ADMM state, integration and
 * source-path buffers.  The serving runtime admits queries by this figure.
 * 0 for NULL mesh, nsrc <= 0 or an unknown formulation. */
uint64_t hg_query_bytes(hg_mesh_t mesh, int32_t nsrc, const hg_opts* opts);

/*
 * The generator loops of the cycle constraints (Sec. 5.1), built with the
 * mesh by a tree-cotree decomposition on the caller's ids: primal tree =
 * breadth-first tree from the smallest vertex of each component (parent =
 * the neighbour one level closer with the smallest id); dual tree =
 * first-in-first-out breadth-first search over faces from the smallest face
 * of each component, edges of a face in slot order, across interior edges
 * not in the primal tree; one loop per interior edge in neither tree, in
 * canonical edge order, on components without boundary.  For such an edge
 * (a, b), a < b:
 *   form HG_FORM_EDGE: a -> b, then back to a through the primal tree;
 *     ids = canonical edge ids, coef = +1 where the loop runs from the
 *     smaller to the larger vertex id, else -1 (1 float per slot);
 *   form HG_FORM_FACE: across the edge from its smaller to its larger face,
 *     then back through the dual tree; ids = caller face ids, coef = the
 *     polyline segment inside the face, from the midpoint of the edge the
 *     loop enters it by to the midpoint of the edge it leaves it by (3
 *     floats per slot).
 *   ptr  : HOST int32[n_cycles + 1] slot offsets of the loops;
 *   ids  : HOST int32[capacity]; coef : HOST float[capacity or 3*capacity].
 * n_cycles and the slot counts are in hg_mesh_stats; HG_E_INVALID_ARG if
 * capacity is below the form's slot count or a pointer is NULL.
 */
hg_status hg_mesh_cycles(hg_mesh_t mesh, int32_t form, int32_t* ptr, int32_t* ids, float* coef,
                         int64_t capacity);

/* ---- the individual steps, each running the same kernels as the solve ---- */

/* Breadth-first sets (Eq. 6): level_dev[v] = hop distance to the source set
 * (-1 if unreachable); parent_dev[v] = the neighbour with level one less and
 * the smallest vertex id (-1 for sources and unreachable vertices).
 * DEVICE int32[nv] outputs (either may be NULL). */
hg_status hg_bfs(hg_mesh_t mesh, const int32_t* src, int32_t nsrc,
                 int32_t* level_dev, int32_t* parent_dev, void* stream, int32_t* depth_out);

/* The same search without allocating device memory, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Arguments, outputs and results are
 * those of hg_bfs.  Its working arrays live in a fixed 64 MiB device array
 * of the library, one per GPU, held from the first call on that GPU until
 * the process ends; it takes meshes of at most 3,000,000 vertices and at
 * most 65,536 sources (HG_E_INVALID_ARG beyond, nothing run).  Calls on
 * one GPU share that array: calls that overlap in time on one GPU (from
 * several threads or on several streams) race and must be serialised by
 * the caller.  The stream is synchronised before returning. */
hg_status hg_bfs_noalloc(hg_mesh_t mesh, const int32_t* src, int32_t nsrc,
                         int32_t* level_dev, int32_t* parent_dev, void* stream, int32_t* depth_out);

/* Diffusion (Eq. 4 by sweeps of Eq. 7): logu_dev = DEVICE float64[nv], the
 * natural log of u (-inf where u = 0).  Uses opts->tol_u / max_sweeps /
 * diffusion_schedule; info receives sweeps, passes, res_u, t. */
hg_status hg_diffuse(hg_mesh_t mesh, const int32_t* src, int32_t nsrc, double t,
                     const hg_opts* opts, double* logu_dev, void* stream, hg_info* info);

/* Normalisation (Eq. 3) from DEVICE float64[nv] log u: h_dev = DEVICE
 * float32[nf*3] unit vectors (0 where the gradient vanishes); on an
 * intrinsic mesh each in its face's own frame, z = 0 (the edge-form ADMM
 * entry point reads it the same way). */
hg_status hg_normalize(hg_mesh_t mesh, const double* logu_dev, float* h_dev, void* stream);

/* Edge-form ADMM (Sec. 4.1) from DEVICE float32[nf*3] normalised field h:
 * x_dev = DEVICE float32[ne] edge differences after `iters` iterations
 * (iters <= 0: run to opts->tol_admm / max_admm).  src/nsrc: HOST source
 * ids or NULL/0; with two or more distinct sources and opts->source_paths
 * the constraints of Eq. 25 are added (paths as in hg_geodesic_solve). */
hg_status hg_admm_edge(hg_mesh_t mesh, const float* h_dev, const int32_t* src, int32_t nsrc, int32_t iters,
                       const hg_opts* opts, float* x_dev, void* stream, hg_info* info);

/* Face-form ADMM (Sec. 3.2): g_dev = DEVICE float32[nf*3] gradients; with
 * sources as above, the constraints of Eq. 24 on the gradient of the face
 * whose counter-clockwise boundary runs each path edge in the path's
 * direction (the only face of a boundary edge). */
hg_status hg_admm_face(hg_mesh_t mesh, const float* h_dev, const int32_t* src, int32_t nsrc, int32_t iters,
                       const hg_opts* opts, float* g_dev, void* stream, hg_info* info);

/* Integration along the breadth-first pairing (Sec. 3.3 / Sec. 4) of edge
 * differences x_dev (float32[ne]) or face gradients g_dev (float32[nf*3]),
 * d_dev = DEVICE float32[nv]. */
hg_status hg_integrate_edge(hg_mesh_t mesh, const int32_t* src, int32_t nsrc,
                            const float* x_dev, float* d_dev, void* stream);
hg_status hg_integrate_face(hg_mesh_t mesh, const int32_t* src, int32_t nsrc,
                            const float* g_dev, float* d_dev, void* stream);

/* Canonical edge list: DEVICE int32[ne*2] (smaller id, larger id). */
hg_status hg_mesh_edges(hg_mesh_t mesh, int32_t* edges_dev, void* stream);

/* The mesh's diffusion weights as computed on the device (Sec. 3.1 and the
 * sweep of Eq. 7): theta_jk = (cot a + cot b)/2 over the edge's one or two
 * faces, written to DEVICE double[ne] in the canonical edge order of
 * hg_mesh_edges, and the lumped vertex area A_j (a third of the areas of
 * the faces around j), written to DEVICE double[nv] in the caller's vertex
 * order.  Either pointer may be NULL (not both).  Synchronises the stream. */
hg_status hg_mesh_weights(hg_mesh_t mesh, double* theta_dev, double* area_dev, void* stream);

/* ---- the comparator of Sec. 6.4: the original heat method by CG ----
 *
 * The paper sets its Gauss-Seidel diffusion and ADMM gradient solver against
 * the original heat method with its direct solves replaced by conjugate
 * gradients with a diagonal preconditioner, measuring the heat residual
 * E_1 = |(A - t L_c) u - u_0|_2 (Eq. 29) and the distance error
 * E_2 = |d - d*|_2 / n (Eq. 30) against time.  These entry points run that
 * CG in FP64 on the device (x0 = 0, Jacobi preconditioner, the CG scalars
 * kept on the device; deterministic reductions).  tol > 0: stop at relative
 * residual |r|/|b| <= tol, checked every 16 iterations, HG_E_NOT_CONVERGED
 * (result written) if max_iters is reached first; tol = 0: exactly
 * max_iters iterations. */
typedef struct {
    int32_t iters;          /* CG iterations run */
    int32_t converged;      /* 1 if the relative residual reached tol */
    double res_rel;         /* final |r|_2 / |b|_2 (recursive residual) */
    double res_abs;         /* final |r|_2 */
    double res_abs0;        /* |b|_2 */
    float ms;               /* device time of the iterations (HIP events) */
    int32_t reserved[3];
} hg_cg_info;

/* CG on Eq. 4, (A - t L_c) u = u_0 with u_0 = 1 at the sources (HOST int32
 * ids), t <= 0 meaning hbar^2.  u_dev = DEVICE float64[nv], plain u (it
 * underflows to 0 where u is below the FP64 range; E_1 is absolute, so the
 * paper's comparison is unaffected). */
hg_status hg_cg_diffuse(hg_mesh_t mesh, const int32_t* src, int32_t nsrc, double t, int32_t max_iters,
                        double tol, double* u_dev, void* stream, hg_cg_info* info);
/* CG on the Poisson step with d = 0 at every source (the paper fixes the
 * source values to make the system definite) from the DEVICE float32[nf*3]
 * normalised field h_dev (caller face order): form HG_FORM_FACE solves
 * K d = r with r_i = sum_f A_f grad phi_i|_f . h_f (Sec. 3.2, the face
 * ADMM's converged answer); HG_FORM_EDGE solves L_E d = b_E (edge weight
 * |H_e|, b_E,i = sum_{f ni i} h_f . (2 p_i - p_j - p_k); the edge ADMM's).
 * d_dev = DEVICE float64[nv]; +inf where no source reaches.  Extrinsic
 * meshes only (HG_E_INVALID_ARG for an intrinsic one). */
hg_status hg_cg_poisson(hg_mesh_t mesh, int32_t form, const float* h_dev, const int32_t* src, int32_t nsrc,
                        int32_t max_iters, double tol, double* d_dev, void* stream, hg_cg_info* info);
/* E_1 of Eq. 29 for the DEVICE float64[nv] field u_dev (is_log = 1: it holds
 * log u, as hg_diffuse writes it), t <= 0 meaning hbar^2; *e1 on the host. */
hg_status hg_heat_residual(hg_mesh_t mesh, const int32_t* src, int32_t nsrc, double t, const double* u_dev,
                           int32_t is_log, double* e1, void* stream);

/* ---- serving: concurrent queries over resident meshes ----
 *
 * A server runs queries on n_slots worker threads, each with its own HIP
 * stream on the device current at creation.  hg_server_submit queues a
 * query and returns at once; a free slot takes the oldest query that can be
 * admitted and runs it exactly as hg_geodesic_solve would (same kernels,
 * private workspace), so results do not depend on what else runs; queries
 * that arrive while others run start as soon as a slot and memory allow and
 * overlap with them on the device.  Admission by device memory: query
 * workspaces are pooled per mesh and reused; a new one is created only while
 * the bytes held stay within workspace_budget (0 = half of the free device
 * memory at creation), releasing idle workspaces of other meshes for the
 * oldest waiting query; with nothing running the oldest query is always
 * admitted.  The bytes held count each workspace at the larger of its
 * admission estimate (hg_query_bytes) and its size after its last query,
 * plus the schedules served queries added to their meshes (face tiles of
 * the blocked edge ADMM, the face form's slot geometry).  Meshes, source arrays' contents (copied at submit) and
 * the output buffers must stay valid until the query's result is taken. */
typedef struct hg_server_s* hg_server_t;

typedef struct {
    int64_t ticket;         /* as returned by hg_server_submit; -1 = none */
    int32_t status;         /* hg_status of the query */
    int32_t reserved0;
    double t_submit, t_start, t_end;   /* hg_server_clock() seconds */
    hg_info info;
} hg_result;

typedef struct {
    int32_t n_slots, pending, running, completed_unread, workspaces_idle;
    int32_t reserved0;
    uint64_t workspace_bytes_held, workspace_bytes_idle, workspace_budget;
    int32_t reserved[8];
} hg_server_stats_t;

/* n_slots in [1, 64].  *out receives the server. */
hg_status hg_server_create(int32_t n_slots, uint64_t workspace_budget, hg_server_t* out);
/* Queue one query: arguments as hg_geodesic_solve (src is copied, opts may be
 * NULL); d_dev is written when the query completes.  *ticket (optional)
 * identifies the result. */
hg_status hg_server_submit(hg_server_t server, hg_mesh_t mesh, const int32_t* src, int32_t nsrc, double t,
                           const hg_opts* opts, float* d_dev, int64_t* ticket);
/* Take the oldest completed result, waiting up to timeout_ms (< 0: without
 * limit); out->ticket = -1 if none completed in time. */
hg_status hg_server_wait(hg_server_t server, hg_result* out, int32_t timeout_ms);
hg_status hg_server_stats(hg_server_t server, hg_server_stats_t* stats);
/* Seconds on the clock of the result timestamps (monotonic). */
double hg_server_clock(void);
/* Runs the queued queries to completion, then frees the server. */
void hg_server_destroy(hg_server_t server);

/* ---- autotuning of the diffusion schedule ---- */
typedef struct {
    int32_t n_candidates;
    int32_t chosen;              /* index into the arrays below */
    int32_t schedule[8];         /* 1 = global Jacobi sweeps, 2 = LDS tiles,
                                    3 = overlapping LDS tiles */
    int32_t inner_sweeps[8];     /* sweeps per tile pass (0 for Jacobi) */
    float ms[8];                 /* time of the diffusion stage (converged) */
    int32_t passes[8];
    int32_t overlap_rings[8];    /* rings of overlap (schedule 3), else 0 */
    int32_t n_admm;              /* ADMM block candidates timed (edge form) */
    int32_t admm_chosen;         /* index into the two arrays below, -1 if none */
    int32_t admm_block[4];       /* iterations per launch */
    float admm_us_per_iteration[4];
} hg_tune_report;

/* Times the diffusion stage of a probe query (src/nsrc, t, opts as in
 * hg_geodesic_solve) once per candidate schedule -- LDS tiles with 16, 32
 * and 64 in-tile sweeps per pass, overlapping LDS tiles with r and r + 1
 * rings (r = opts->overlap_rings, 1 if 0) and 32 or 64 sweeps, and global
 * Jacobi sweeps on meshes of at most 16 tiles -- on the mesh's default
 * workspace and stream, and stores
 * the fastest one that converges in the mesh: later queries whose
 * diffusion_schedule / inner_sweeps options are 0 (auto) use it.  The
 * arithmetic of every candidate has the same fixed point.  For the edge form
 * with opts->admm_block 0 it then times 192 ADMM iterations (runs of 64, as
 * between two checks of a solve) in launches of 4, 5 and 6 iterations over
 * LDS face tiles and stores the fastest block for later queries with
 * admm_block 0; every block gives the same iterates.  Overlapping tiles and
 * face tiles built for the trials are kept only if they are chosen.  The
 * call changes the mesh: it must not run while other calls use the same
 * mesh.  report (optional) receives the timings. */
hg_status hg_mesh_autotune(hg_mesh_t mesh, const int32_t* src, int32_t nsrc, double t, const hg_opts* opts,
                           void* stream, hg_tune_report* report);

/* Thread-local message of the last failing call ("" if none). */
const char* hg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HGEO_H */
