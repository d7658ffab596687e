/*
 * pamo.h -- C ABI of the MI355X (gfx950) implementation of parallel,
 * intersection-free QEM edge-collapse mesh simplification, the simplification
 * stage of PaMO (Oh, Yuan, Wei, Shi, Xiang, Liu, Su; Pacific Graphics 2025):
 * Sec. 5, the "Parallel Intersection-Free Mesh Simplification" algorithm,
 * Eq. 1, Sec. 5.2 and Appendix 3 (self-intersection test), Sec. 5.3 (undo,
 * invalid flags, tolerance).
 *
 * Conventions for every entry point
 *   - Mesh arrays are DEVICE pointers on the context's device, allocated and
 *     owned by the caller: V is float64 [nv][3], F is int32 [nf][3] with the
 *     corners counter-clockwise seen from outside.  The input must be a closed
 *     (watertight) edge- and vertex-manifold mesh without exactly degenerate
 *     triangles, every vertex used by some face, and free of
 *     self-intersections -- the output of the paper's remeshing stage (Sec. 3
 *     and 4).  Coordinates are expected in [0,1]^3 (Sec. 3 normalises the
 *     input there; the default weights of Eq. 1 assume that scale).
 *   - Half-edge h = 3 f + c runs from F[f][c] to F[f][(c+1)%3].  An edge is
 *     named by its smaller half-edge id.
 *   - All work is enqueued on the context's stream.  Functions that return
 *     host-visible counts synchronise that stream before returning; the others
 *     are asynchronous and write their counts to device memory.
 *   - Return value: 0 success, 1 PAMO_TARGET_UNREACHED (warning), < 0 error;
 *     pamo_last_error() then describes it.  No C++ exception crosses this
 *     boundary.  After an error the outputs are unspecified; inputs are never
 *     modified unless the entry point says so.
 *   - One context per host thread; calls on one context must not overlap.
 */
#ifndef PAMO_H
#define PAMO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pamo_ctx pamo_ctx;
typedef int32_t pamo_status;

#define PAMO_OK 0
#define PAMO_TARGET_UNREACHED 1   /* stopped after `tolerance` rounds without a collapse (Sec. 5.3) */
#define PAMO_ERR_ARG (-1)         /* bad argument (null pointer, size, index out of range) */
#define PAMO_ERR_NONMANIFOLD (-2) /* open, non-manifold, inconsistently oriented or with unused vertices */
#define PAMO_ERR_SELF_INTERSECTING (-3) /* input has a self-intersection (only when validating) */
#define PAMO_ERR_DEGENERATE (-4)  /* a face repeats a vertex */
#define PAMO_ERR_HIP (-6)         /* HIP runtime error */
#define PAMO_ERR_CAPACITY (-7)    /* an internal bound was exceeded (traversal stack, deferred pairs), or
                                     the caller's workspace is too small (pamo_set_workspace) */

typedef struct {
  double w_e;          /* edge-length weight of Eq. 1 (paper default 0.001) */
  double w_s;          /* skinny-triangle weight of Eq. 1 (paper default 0.005) */
  int32_t tolerance;   /* zero-collapse rounds before giving up (paper default 4, Sec. 5.3) */
  int32_t max_rounds;  /* stop after this many rounds (< 0: no limit) */
  int32_t validate_input; /* 1: check manifoldness and self-intersections of the input first */
  /* tuning knobs: none changes a result; 0 selects the library default */
  int32_t query_packet; /* queries walking the BVH together, one lane each (1,2,4,8,16,32,64; default 1) */
  int32_t resort_every; /* re-sort the BVH leaves by Morton code every this many rounds (default: never;
                           the first round's order is carried through the compactions) */
  int32_t query_coop;   /* lanes sharing one query when few queries remain (2,4,8,16; 1 = never; default 8) */
  int32_t coop_below;   /* ... namely when a pass has fewer than about this many queries (default 65536) */
  int32_t learned;      /* 1: the learned proposal (needs pamo_set_mlp); 0: the plain method */
  double cost_target;   /* > 0: target-cost termination (the paper ends a run at a target edge cost or a
                           target face count, Sec. 5.1 "Edge Collapse"): only edges whose Eq. 1 cost is at
                           most this are collapsed, and a round that selects no edge ends the run with
                           PAMO_OK (the face target still applies; pass 0 faces for cost alone).
                           <= 0: off (default) */
  int32_t prefilter;    /* 1: the local checks (link condition, degenerate or flipped generated triangles;
                           Sec. 5.1 applies the link condition during the collapse) run on every keyed edge
                           before the selection, and an edge failing them gets no key that round, so it does
                           not hold back its neighbourhood (the other order of selection and local checks);
                           0: checks on the selected candidates only (default).  Applies to pamo_simplify,
                           pamo_simplify_batch and pamo_select; pamo_collect refuses it (PAMO_ERR_ARG) */
  int32_t key_mode;     /* 0: the 64-bit key of Sec. 5.1 "Cost Propagation", float32 cost code above the edge
                           id (default); 1: edges ordered by the float64 cost, then the edge id (the other
                           reading of the paper's conversion of costs from floats): each keyed edge's key is
                           its rank in that order above its id.  The learned proposal, pamo_features and
                           pamo_collect read the float32 cost from the key and refuse it (PAMO_ERR_ARG) */
  int32_t pair_capacity; /* first capacity (pairs) of a query pass's candidate-pair buffer; a pass that
                           collects more grows the buffer and runs again (no effect on results).
                           0: max(2^20, 16 nf) (default) */
} pamo_options;

typedef struct {
  int64_t rounds;       /* rounds run */
  int64_t faces_out, verts_out;
  int64_t candidates;   /* independent-region edges selected, summed over rounds */
  int64_t commits;      /* collapses kept */
  int64_t rej_link;     /* rejected by the link condition */
  int64_t rej_flip;     /* rejected: a generated triangle degenerate or flipped */
  int64_t rej_isect;    /* undone because of a self-intersection */
  int64_t capped;       /* passed but not needed to reach the exact target */
  int64_t undo_hist[5]; /* rounds needing 0, 1, 2, 3, >3 undo iterations (cf. Table 7) */
  int64_t deferred_pairs; /* pairs settled by the exact (expansion) predicate */
  int64_t status;       /* as the return value */
  int64_t demoted;      /* learned proposal: candidates set aside by the network */
  int64_t fallbacks;    /* learned proposal: rounds run again without it (nothing committed) */
} pamo_stats;

/* Fill *opt with the paper's defaults (w_e 0.001, w_s 0.005, tolerance 4). */
void pamo_default_options(pamo_options* opt);

/* Create a context on `device` that enqueues on `hip_stream` (a hipStream_t;
 * NULL = the null stream).  `opt` may be NULL (defaults).  Unless it is given
 * a workspace (pamo_set_workspace), the context allocates its own device
 * workspace, which grows to fit the largest mesh seen. */
pamo_status pamo_create(pamo_ctx** out, int device, void* hip_stream, const pamo_options* opt);
void pamo_destroy(pamo_ctx* ctx);
pamo_status pamo_set_options(pamo_ctx* ctx, const pamo_options* opt);
/* Message of the last error on this context (valid until the next call). */
const char* pamo_last_error(const pamo_ctx* ctx);

/* Device workspace (scratch) of the method (the problem statement of Sec. 3:
 * a mesh in, its simplification out; everything between lives here).
 *
 * pamo_workspace_bytes: bytes of workspace that suffice for every mesh entry
 * point (pamo_quadrics, pamo_select, pamo_check, pamo_collapse,
 * pamo_simplify, pamo_simplify_batch with up to 4096 meshes of these totals,
 * pamo_collect, pamo_features, pamo_self_intersections) on a mesh of nv
 * vertices and nf faces with options opt (NULL: defaults): the exact sum of
 * the buffers those calls reserve, each rounded up to 256 bytes.  A query
 * pass whose candidate pairs overflow pair_capacity takes more, when the
 * workspace has it, and fails with PAMO_ERR_CAPACITY when it has not.
 * Returns 0 for sizes no entry point accepts (nv or nf below 4, nf above
 * 2^31 / 3).  Host-only; no context or device needed.
 *
 * pamo_set_workspace: from now on the context takes all its device scratch
 * from dev (device memory on the context's device, 256-byte aligned, at least
 * 4 KiB, owned by the caller, e.g. a torch tensor), which the caller keeps
 * alive and leaves alone while calls on the context run; every call carves it
 * afresh from its start, so nothing in it outlives a call.  The context frees
 * the workspace it allocated before.  A call whose needs exceed `bytes` fails
 * with PAMO_ERR_CAPACITY (the message names the buffer); the mesh entry points
 * fit whenever bytes >= pamo_workspace_bytes(nv, nf, opt).  The remeshing and
 * training entry points carve what they need as they go.  dev = NULL: back to
 * workspace the context allocates itself.  Synchronises the stream.
 *
 * pamo_workspace_held: bytes of device workspace the context has allocated
 * itself and holds (0 while it works in a caller's workspace). */
size_t pamo_workspace_bytes(int64_t nv, int64_t nf, const pamo_options* opt);
pamo_status pamo_set_workspace(pamo_ctx* ctx, void* dev, size_t bytes);
int64_t pamo_workspace_held(const pamo_ctx* ctx);

/* ---- round-level steps (stateless: the caller owns everything between calls) ---- */

/* Per-vertex quadric error metric (Garland-Heckbert, named for the Q_ab term of
 * Eq. 1): Q[v] = sum over the faces around v, in ascending face slot, of the
 * plane quadric of the face (unit normal n, offset d = -n.p0), stored as the
 * 10 entries xx xy xz xw yy yz yw zz zw ww.  Q: device float64 [nv][10]. */
pamo_status pamo_quadrics(pamo_ctx* ctx, const double* V, int64_t nv, const int32_t* F, int64_t nf, double* Q);

/* Edge costs (Eq. 1 with the QEM placement), 64-bit keys and the independent
 * edges of one round (cost propagation and region selection of Sec. 5.1).
 * The quadrics are recomputed from V and F inside (they are a pure function
 * of the mesh; a caller's Q could only disagree), so no Q is taken.
 *   flags  device uint8 [3 nf] invalid-edge flags, or NULL
 *   demote device uint8 [3 nf] edges to leave out this round, or NULL
 *   keys   device uint64 [3 nf] output (key of the edge on both half-edges;
 *          UINT64_MAX for flagged edges), or NULL
 *   cand   device int32, capacity 3 nf: chosen edges (smaller half-edge id), ascending
 *   ncand  device int32 [1]: their number
 * Asynchronous. */
pamo_status pamo_select(pamo_ctx* ctx, const double* V, int64_t nv, const int32_t* F, int64_t nf,
                        const uint8_t* flags, const uint8_t* demote, uint64_t* keys, int32_t* cand,
                        int32_t* ncand);

/* Check the chosen edges of one round: link condition (Sec. 5.1), exact
 * degeneracy and normal flip of the generated triangles, the exact face
 * target (keep the smallest keys when more pass than needed to reach
 * target_faces), then apply them together to an internal copy and run the
 * intersection check / undo loop (Sec. 5.2, 5.3) to its fixed point.
 *   cand, ncand  as produced by pamo_select for the same V, F, flags (at most
 *                nf / 2 + 1 of them: chosen edges have disjoint rings)
 *   vbar   device float64 [ncand][3] output: new vertex position
 *   reason device uint8 [ncand] output: 0 collapse, 1 link condition,
 *          2 degenerate or flipped triangle, 3 self-intersection, 4 not needed
 * V and F are not modified.  Synchronises the stream. */
pamo_status pamo_check(pamo_ctx* ctx, const double* V, int64_t nv, const int32_t* F, int64_t nf,
                       const uint8_t* flags, int64_t target_faces, const int32_t* cand, const int32_t* ncand,
                       double* vbar, uint8_t* reason, int64_t* undo_iterations);

/* Commit the collapses with reason 0 and compact the mesh IN PLACE (stable:
 * surviving vertices and faces keep their relative order).  Also writes the
 * invalid-edge flags for the next round into flags_io (device uint8 [3 nf] in,
 * [3 nf_out] out, may be NULL): the edges rejected with reason 1-3, plus the
 * previous flags when nothing was committed (Sec. 5.3).  *nv and *nf (host)
 * are updated.  Synchronises the stream. */
pamo_status pamo_collapse(pamo_ctx* ctx, double* V, int64_t* nv, int32_t* F, int64_t* nf, const int32_t* cand,
                          const int32_t* ncand, const double* vbar, const uint8_t* reason, uint8_t* flags_io);

/* ---- the whole method ---- */

/* Simplify until exactly target_faces - (target_faces mod 2) faces remain, or
 * `tolerance` rounds in a row collapse nothing (returns PAMO_TARGET_UNREACHED
 * with the mesh reached), or max_rounds.  V_out / F_out: device buffers of at
 * least nv / nf rows; *nv_out, *nf_out host.  stats (host) may be NULL.
 * Synchronises the stream. */
pamo_status pamo_simplify(pamo_ctx* ctx, const double* V, int64_t nv, const int32_t* F, int64_t nf,
                          int64_t target_faces, double* V_out, int64_t* nv_out, int32_t* F_out, int64_t* nf_out,
                          pamo_stats* stats);

/* pamo_simplify for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same method, arguments and results as pamo_simplify, but every buffer
 * of the call lives in one static device array of PAMO_NOALLOC_SCRATCH_BYTES
 * that each GPU the library runs on holds from the library's load until the
 * process ends; the call allocates no device memory and no pinned host memory
 * (no hipMalloc, hipFree or hipHostMalloc) and creates no HIP events (only
 * the host bookkeeping of its buffer table uses the C++ heap); the context
 * must have been created (pamo_create finds the array's device address).  A
 * mesh whose buffers do not fit fails
 * with PAMO_ERR_CAPACITY before any work (at the default options a closed
 * mesh needs about 950 bytes per face, so meshes up to about 140,000 faces
 * fit; pamo_workspace_bytes gives the size of a larger workspace for
 * pamo_simplify).  Every call on a GPU shares that
 * GPU's array and leaves its contents behind: calls that overlap on one GPU,
 * from any context or thread, race and must not be made.  Synchronises the
 * stream. */
#define PAMO_NOALLOC_SCRATCH_BYTES (128u << 20)
pamo_status pamo_simplify_noalloc(pamo_ctx* ctx, const double* V, int64_t nv, const int32_t* F, int64_t nf,
                                  int64_t target_faces, double* V_out, int64_t* nv_out, int32_t* F_out,
                                  int64_t* nf_out, pamo_stats* stats);

/* The batched form: simplify nmesh independent meshes together.  The meshes
 * are concatenated into one set of arrays and every kernel launch of a round
 * covers all of them, so a batch of small meshes fills the GPU the way one
 * large mesh does (small meshes alone gain little from the parallel method,
 * as the paper's Limitations section observes).  Each mesh receives exactly
 * the result pamo_simplify gives it alone: the same rounds, output and
 * statistics.
 *   nmesh        1 .. 4096
 *   V, F         device, the meshes concatenated: float64 [v_off[nmesh]][3]
 *                and int32 [f_off[nmesh]][3]; F holds vertex ids local to
 *                its mesh (0 .. nv of the mesh - 1)
 *   v_off, f_off host int64 [nmesh + 1]: mesh m owns vertex rows
 *                v_off[m] .. v_off[m+1]-1 and face rows f_off[m] .. f_off[m+1]-1;
 *                v_off[0] = f_off[0] = 0; every mesh has >= 4 vertices and faces
 *   targets      host int64 [nmesh]: face target of each mesh
 *   V_out, F_out device, at least v_off[nmesh] / f_off[nmesh] rows: the
 *                simplified meshes concatenated in the same order, local ids
 *   v_out_off, f_out_off host int64 [nmesh + 1] output: where each output
 *                mesh lies in V_out / F_out
 *   stats        host pamo_stats [nmesh], or NULL; deferred_pairs holds the
 *                batch total in every entry (the exact pass is shared)
 * Returns PAMO_TARGET_UNREACHED when any mesh stopped early (its stats.status
 * tells which), else PAMO_OK; errors as pamo_simplify, about any of the meshes.
 * Coordinates outside [0,1]^3 stay correct but cost speed (the BVH gives each
 * mesh the cell [0,1]^3 of its own).  Synchronises the stream. */
pamo_status pamo_simplify_batch(pamo_ctx* ctx, int32_t nmesh, const double* V, const int64_t* v_off,
                                const int32_t* F, const int64_t* f_off, const int64_t* targets, double* V_out,
                                int64_t* v_out_off, int32_t* F_out, int64_t* f_out_off, pamo_stats* stats);

/* ---- remeshing (the stage before the path), mesh-to-volume step ---- */

/* The unsigned distance field of a triangle soup in a narrow band (Sec. 4.1,
 * Mesh-to-Volume): at the centre ((i + 1/2) / res, (j + 1/2) / res,
 * (k + 1/2) / res) of every voxel of a res^3 grid over [0,1]^3,
 * udf[(i * res + j) * res + k] = the smallest float64 distance from the centre
 * to any triangle of (V, F) when it is at most `band`, else +infinity (the
 * paper keeps a band of 3 / res).  V: device float64 [nv][3], F: device int32
 * [nf][3] (any soup: no manifoldness or orientation is assumed; nf may be 0);
 * udf: device float64 [res^3], written whole.  res in [1, 2048], band > 0.
 * Fails with PAMO_ERR_ARG on an index outside [0, nv), and with
 * PAMO_ERR_CAPACITY (udf then holds no field) when one
 * triangle's banded box covers more than 2^20 tiles of 4^3 voxels, when nf
 * exceeds 2^26, or when the (tile, triangle) pairs that pass the band filter
 * exceed 2^26 in all (the per-triangle counts and the pairs are scanned whole).
 * Synchronises the stream. */
pamo_status pamo_udf(pamo_ctx* ctx, const double* V, int64_t nv, const int32_t* F, int64_t nf, int32_t res,
                     double band, double* udf);

/* ---- remeshing, volume-to-mesh step ---- */

/* Dual Marching Cubes (Sec. 4.2, Volume-to-Mesh) on a res^3 grid of values
 * S[(i * res + j) * res + k] (device float64) at the points ((i + 1/2) / res,
 * (j + 1/2) / res, (k + 1/2) / res); a point is outside when S - iso >= 0.
 * Per cube of 2^3 points: one vertex per surface patch, at the mean of the
 * crossing points of its edges: at the fraction t = s0 / (s0 - s1) of an edge
 * when beta = 0, at 1 / (1 + exp(-beta (t - 1/2))) when beta > 0 (Appendix
 * 2.1's smoothing, beta = 5 in the paper); patches come from face links, and an
 * ambiguous face shared by two cubes that would otherwise give a non-manifold
 * dual edge is resolved the other way in both (the paper's manifold fix).
 * Per crossed grid edge with four neighbouring cubes: one quad, oriented with
 * its normal towards the outside, divided by the envelope of the grid edge
 * (Appendix 2.1): with p+ and p- the edge's positive and negative ends and l,
 * r a quad vertex v's neighbours, v is concave when
 * (v - p+) . ((l - p+) x (r - p+)) < 0 or (v - p-) . ((l - p-) x (r - p-)) > 0;
 * concave vertices on one diagonal only: two triangles split along it; on
 * both: four triangles around an extra vertex at the edge's (smoothed)
 * crossing point; none: the two triangles whose smallest angle is larger.
 * Vertices are numbered by cube (x outermost) then patch, then the extra
 * edge vertices in quad order; faces by axis then grid point, two or four per
 * quad.  V_out: device float64 [vcap][3]; F_out: device int32 [fcap][3];
 * *nv_out, *nf_out (host) get the sizes.  res in [2, 512], at most 2^26 cubes
 * crossed by the surface and 2^26 quads (else PAMO_ERR_HIP); values must be
 * finite where a sign change occurs.  Fails with PAMO_ERR_CAPACITY, writing
 * only the sizes, when the mesh does not fit, and PAMO_ERR_ARG for beta < 0 or
 * not finite.  Synchronises the stream. */
pamo_status pamo_dualmc(pamo_ctx* ctx, const double* S, int32_t res, double iso, double beta, double* V_out,
                        int64_t vcap, int32_t* F_out, int64_t fcap, int64_t* nv_out, int64_t* nf_out);

/* ---- safe projection (the stage after the path), Sec. 6 ---- */

/* Options of the safe projection; pamo_project_defaults gives the paper's
 * values (Sec. 6.1, Sec. 6.2: k_dis 1e3, k_elas 1e-1, k_bend 1e-2, k_bar 1e2,
 * dhat 1e-3, T = 50 iterations, targets refreshed every 10) and this
 * library's choices where the paper gives none (CG tolerance 1e-4 relative
 * to |grad B|, at most 1000 CG iterations; additive CCD keeps 0.1 of each
 * pair's distance; at most 40 line-search halvings). */
typedef struct {
  double k_dis, k_elas, k_bend, k_bar;
  double dhat;
  double cg_tol;
  double accd_s;
  int32_t iterations;
  int32_t refresh;
  int32_t cg_max;
  int32_t ls_max;
} pamo_project_options;

typedef struct {
  int32_t iterations;  /* iterations run */
  int32_t cg_iters;    /* CG iterations, summed */
  int32_t halvings;    /* line-search halvings, summed */
  int32_t stalled;     /* iterations whose line search found no decrease of B */
  int64_t max_pt, max_ee;  /* most point-triangle / edge-edge contacts at an iteration's start */
  double B_first, B_last;  /* B at the first iteration's start and at the end */
} pamo_project_stats;

void pamo_project_defaults(pamo_project_options* opt);

/* Uniform samples on a triangle mesh (the m points of E_M2S, Sec. 6.1): from
 * uniforms U (device float64 [m][3] in [0, 1)), sample s lies on the first
 * triangle whose inclusive cumulative area exceeds U[s][0] times the total,
 * at (1 - r) a + r (1 - U[s][2]) b + r U[s][2] c with r = sqrt(U[s][1])
 * (uniform on the triangle).  Y: device float64 [m][3].  *area (host, may be
 * NULL) gets the total area.  Synchronises the stream. */
pamo_status pamo_sample_surface(pamo_ctx* ctx, const double* V, int64_t nv, const int32_t* F, int64_t nf,
                                const double* U, int64_t m, double* Y, double* area);

/* The closest-feature targets of App. 2.2 for the mesh (X, F) being projected
 * towards (Vin, Fin): targets[i] (device float64 [nv][3]) the point of the
 * input mesh closest to X[i]; tri[s] (device int32 [m]) the triangle of (X, F)
 * closest to the sample Y[s] (device float64 [m][3]).  Ties go to the smallest
 * triangle index whose squared distance is within a relative 1e-9 of the
 * smallest.  Synchronises the stream. */
pamo_status pamo_project_targets(pamo_ctx* ctx, const double* X, int64_t nv, const int32_t* F, int64_t nf,
                                 const double* Vin, int64_t nv_in, const int32_t* Fin, int64_t nf_in, const double* Y,
                                 int64_t m, double* targets, int32_t* tri);

/* The pieces of one iteration of Alg. 2 at positions X (device [nv][3]) of the
 * mesh F (device int32 [nf][3], closed and manifold) with rest shape X0, the
 * given targets and tri (as pamo_project_targets writes them), samples Y and
 * input area area_in (the weight A_in / m of E_M2S).  parts (host [6]): the
 * unweighted terms E_S2M, E_M2S, E_elas, E_bend, the barrier sum, then B;
 * contacts (host [2], may be NULL): point-triangle and edge-edge pairs closer
 * than dhat.  Optional (NULL to skip), all device [nv][3]: grad = grad B; Hv =
 * H v for the element-wise projected Hessian H; dir = the CG solution of
 * H p = -grad B (with *cg_iters, host) and *step (host) the additive-CCD step
 * bound along it.  Synchronises the stream. */
pamo_status pamo_project_eval(pamo_ctx* ctx, const double* X0, const double* X, int64_t nv, const int32_t* F,
                              int64_t nf, const double* targets, const double* Y, const int32_t* tri, int64_t m,
                              double area_in, const pamo_project_options* opt, double* parts, int64_t* contacts,
                              double* grad, const double* v, double* Hv, double* dir, int32_t* cg_iters, double* step);

/* Safe projection (Sec. 6, Alg. 2; App. 2.2): moves the vertices of the
 * simplified mesh (Vs, Fs: device, closed, manifold, free of
 * self-intersections) towards the input mesh (Vin, Fin: device, any triangle
 * mesh) by projected Newton on B = k_dis (E_S2M + E_M2S) + k_elas E_elas +
 * k_bend E_bend + k_bar sum b(d): per iteration the element Hessians are
 * projected to positive semi-definite, the direction comes from conjugate
 * gradients, additive CCD bounds the step so that no pair of primitives meets
 * along it, and the step is halved until B decreases.  Y: device float64
 * [m][3], the samples of E_M2S on the input mesh (pamo_sample_surface).
 * V_out: device float64 [nv][3] (may equal Vs).  log (host, may be NULL):
 * [iterations][8] per iteration: B at its start, the CCD bound, the step
 * taken (0 when none decreased B), halvings, CG iterations, point-triangle
 * and edge-edge contacts, |grad B|.  Fails with PAMO_ERR_NONMANIFOLD when
 * (Vs, Fs) is not a closed oriented manifold.  Synchronises the stream. */
pamo_status pamo_safe_project(pamo_ctx* ctx, const double* Vs, int64_t nv, const int32_t* Fs, int64_t nf,
                              const double* Vin, int64_t nv_in, const int32_t* Fin, int64_t nf_in, const double* Y,
                              int64_t m, const pamo_project_options* opt, double* V_out, double* log,
                              pamo_project_stats* stats);

/* ---- utilities ---- */

/* All pairs (t < u) of faces that intersect under the test of Sec. 5.2 /
 * Appendix 3 with exact signs.  pairs: device int32 [cap][2]; *npairs (host)
 * gets the total, which may exceed cap (then only cap pairs are written, in
 * no particular order).  Also fails with PAMO_ERR_NONMANIFOLD on an invalid mesh.
 * Synchronises the stream. */
pamo_status pamo_self_intersections(pamo_ctx* ctx, const double* V, int64_t nv, const int32_t* F, int64_t nf,
                                    int32_t* pairs, int64_t cap, int64_t* npairs);

/* Evaluate the pair test on n explicit triangle pairs: P, Q device float64
 * [n][9] (corner positions), ip, iq device int32 [n][3] (vertex ids, which
 * decide the shared-vertex case), out device uint8 [n] (1 = intersect).
 * Asynchronous. */
pamo_status pamo_tri_pairs(pamo_ctx* ctx, const double* P, const int32_t* ip, const double* Q, const int32_t* iq,
                           int64_t n, uint8_t* out);

/* ---- the learned proposal (an addition to the paper's method) ----
 *
 * Entry points: pamo_set_mlp (set the network's weights), pamo_mlp_logits
 * (inference), pamo_mlp_grad and pamo_mlp_train (training: gradient, and Adam
 * steps over many batches in one call), plus pamo_features and pamo_collect
 * (the training rows).  Training takes float master weights and a batch
 * schedule rather than one bfloat16 step per call, so that thousands of
 * steps run without a host round trip; inference takes the grid-exact
 * network of pamo_mlp below.
 *
 * Each round, a small network scores every selected candidate from 32
 * features of its neighbourhood; candidates scored below a threshold are set
 * aside for the round (their key becomes the largest) and the selection is
 * redone, so a neighbour of a likely rejection can collapse instead.  Every
 * collapse still passes every check of Sec. 5.1 and 5.2.  A round that sets
 * candidates aside and commits nothing runs again without the network.  The
 * network is consulted only in rounds that follow a round whose checks
 * rejected at least one candidate (per mesh in a batch; the first round is
 * plain): where nothing is rejected it has nothing to predict.
 *
 * Features of edge (a, b), each scaled by a fixed power of two and rounded to
 * an integer in [-127, 127]; S = star(a) u star(b), spokes = edges of S's
 * faces through a or b:
 *   0 plog2(cost of Eq. 1) (x4)   1 plog2(length) (x8)   2 length / longest spoke (x128)
 *   3 shortest spoke / length (x128)   4 cos between the normals of the edge's faces (x64)
 *   5 smallest such cos over the spokes (x64)   6, 7 valence of a, b (x4)
 *   8 common neighbours of a and b (x16)   9 sum over S of ovl (x1)   10 largest ovl over S (x4)
 *   11..31 zero
 * plog2(c) = e - 1 + (2 m - 1) for c = m 2^e, m in [0.5, 1) (exact at powers
 * of two, linear between); ovl(f) = alive faces sharing no vertex with f whose
 * float64 boxes meet f's (closed), counted on the input and, for each face a
 * round changes, on that round's tentative mesh, kept when the collapse is
 * committed.
 *
 * Network: 32 -> 64 -> 64 -> 1 with ReLU; each hidden activation h is
 * replaced by min(127, rint(h 2^a)).  Weights of layer l are integers k,
 * |k| <= 127, times 2^-e_l; biases integers times 2^-e_l with magnitude at
 * most 2^22 2^-e_l; 0 <= e_l <= 15.  Under these grids every operation of the
 * inference is exact in float32, so results do not depend on summation order. */
typedef struct {
  float w1[64][32]; /* w1[j][k]: feature k -> unit j */
  float b1[64];
  float w2[64][64];
  float b2[64];
  float w3[64];
  float b3;
  int32_t e1, e2, e3; /* weight grids 2^-e */
  int32_t a1, a2;     /* activation shifts */
  float threshold;    /* set aside when the logit is below */
} pamo_mlp;

/* Set the network of the learned proposal (host struct, copied); NULL
 * removes it.  PAMO_ERR_ARG when a value is off its grid. */
pamo_status pamo_set_mlp(pamo_ctx* ctx, const pamo_mlp* mlp);

/* Features (as above) of the edges given by half-edge ids (device int32
 * [ne]) of a mesh, with the overlap counts of the mesh itself.  X: device
 * float [ne][32]; ovl: device int32 [nf] or NULL.  Synchronises the stream. */
pamo_status pamo_features(pamo_ctx* ctx, const double* V, int64_t nv, const int32_t* F, int64_t nf,
                          const int32_t* edges, int64_t ne, float* X, int32_t* ovl);

/* The network's logit of each feature row: X device float [n][32] (integers
 * in [-127, 127]), logits device float [n].  Asynchronous. */
pamo_status pamo_mlp_logits(pamo_ctx* ctx, const float* X, int64_t n, float* logits);

/* The plain method on one mesh, logging one training row per candidate that
 * a check decided (committed: label 1; rejected by the link condition, a
 * flipped or degenerate triangle, or an intersection: label 0), in round and
 * candidate order: features X device float [cap][32], labels y device uint8
 * [cap]; *rows (host) = rows written.  Synchronises the stream. */
pamo_status pamo_collect(pamo_ctx* ctx, const double* V, int64_t nv, const int32_t* F, int64_t nf,
                         int64_t target_faces, float* X, uint8_t* y, int64_t cap, int64_t* rows, pamo_stats* stats);

/* Training of the network on feature rows X (device float [n][32]) and labels
 * y (device uint8 [n]).  params: device float [6337], the float master
 * weights in the order W1 (64 x 32, row = unit) | b1 | W2 (64 x 64) | b2 | W3 |
 * b3; meta (host int32 [5]): e1, e2, e3, a1, a2.  The forward pass rounds the
 * master weights to their grids; gradients pass straight through every
 * rounding (zero where a value is clamped).  Loss: mean binary cross-entropy
 * of the logit.
 * pamo_mlp_grad: gradient (device float [6337]) and loss (host) over all n rows.
 * pamo_mlp_train: `steps` Adam steps (beta 0.9, 0.999, eps 1e-8, rate lr) on
 * batches of `batch` rows order[s * batch .. (s+1) * batch) (device int32
 * [steps * batch]; entries outside [0, n) are left out of their batch); m, v
 * device float [6337] Adam moments; t0 = steps taken before; loss device
 * float [steps] or NULL.  Asynchronous. */
pamo_status pamo_mlp_grad(pamo_ctx* ctx, const float* params, const int32_t* meta, const float* X, const uint8_t* y,
                          int64_t n, float* grad, float* loss);
pamo_status pamo_mlp_train(pamo_ctx* ctx, float* params, float* m, float* v, const int32_t* meta, const float* X,
                           const uint8_t* y, int64_t n, const int32_t* order, int64_t steps, int64_t batch, float lr,
                           int64_t t0, float* loss);

/* One-sided Hausdorff distance from points P (device float64 [np][3]) to the
 * surface (V, F): dist (device float64 [np], may be NULL) gets each point's
 * distance to its closest triangle, *dmax (host) the largest.  Brute force
 * over the triangles.  Synchronises the stream. */
pamo_status pamo_hausdorff(pamo_ctx* ctx, const double* P, int64_t np, const double* V, int64_t nv, const int32_t* F,
                           int64_t nf, double* dist, double* dmax);

/* ---- measurement ---- */

/* Time phases of the round driver with HIP events on the context stream.
 * Bit i of phase_mask enables phase i (0 disables all).  Each timed launch
 * also adds its algorithmic byte count: the bytes the phase must move at
 * minimum for the mesh size it ran on (every input read once, every output
 * written once).  Host-only bookkeeping; no effect on results. */
pamo_status pamo_profile_enable(pamo_ctx* ctx, uint32_t phase_mask);
/* Number of phases and the name of phase i ("" when out of range). */
int32_t pamo_profile_phases(void);
const char* pamo_profile_name(int32_t phase);
/* Totals since the last reset: launches, milliseconds (HIP event elapsed
 * time), algorithmic bytes.  Synchronises the stream. */
pamo_status pamo_profile_read(pamo_ctx* ctx, int32_t phase, int64_t* launches, double* ms, double* bytes);
pamo_status pamo_profile_reset(pamo_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* PAMO_H */
