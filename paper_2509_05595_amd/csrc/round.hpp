// Launch wrappers of the round kernels and the LBVH (internal).
#pragma once
#include "internal.hpp"

// error bits raised by kernels into one device int
#define PAMO_EBIT_INDEX 1        // vertex index out of range
#define PAMO_EBIT_DEGENERATE 2   // a face repeats a vertex
#define PAMO_EBIT_EDGE 4         // an edge without exactly two faces
#define PAMO_EBIT_ORIENT 8       // the two faces of an edge run the same way
#define PAMO_EBIT_VERTEX 16      // unused vertex, or a vertex star that is not one fan
#define PAMO_EBIT_RING 32        // a vertex star longer than the walk guard
#define PAMO_EBIT_STACK 64       // BVH traversal stack overflow
#define PAMO_EBIT_DEFER 128      // deferred exact-pair list overflow
#define PAMO_EBIT_TILES 256      // a triangle of the distance field reaches too many tiles

namespace pamo {

struct MeshView {
  double* V;
  int* F;
  int* twin;
  int* vh;
  uint8_t* flags;
  int nv, nf;
  int* fmesh = nullptr;  // batches only: mesh of each face / vertex (kept through compaction)
  int* vmesh = nullptr;
  int* ovl = nullptr;    // learned proposal only: per-face overlap counts (kept through compaction)
  // per-round vertex data written by the quadrics kernel when set (not carried
  // through compaction): the half-edges leaving each vertex, ascending (so its
  // star faces h / 3 are ascending too, and h % 3 is the vertex's corner in
  // each; VSTAR per vertex, INT_MAX padding), its star size, and the box of
  // its closed 1-ring (lo, hi)
  int* vstar = nullptr;
  int* vdeg = nullptr;
  double* vbox = nullptr;
};
constexpr int VSTAR = 16;

// Batches keep their meshes apart in the BVH by shifting each mesh's boxes
// to its own cell of a 16 x 16 x 16 grid of pitch 2 (meshes live in [0,1]^3).
__host__ __device__ __forceinline__ void mesh_shift(int m, double& ox, double& oy, double& oz) {
  ox = 2.0 * (m & 15);
  oy = 2.0 * ((m >> 4) & 15);
  oz = 2.0 * (m >> 8);
}
constexpr int PAMO_MAX_MESHES = 4096;

// reserve the round kernels' own buffers for a mesh (or batch of nmesh
// meshes, nmesh > 1) of nv vertices and nf faces, with at most ncand
// candidates per round; key_mode: the float64 key mode's ranking buffers
void round_reserve(Workspace& ws, int64_t nv, int64_t nf, int64_t ncand, int nmesh, bool key_mode);
void launch_adjacency(Workspace& ws, hipStream_t s, MeshView m, int* err);
void launch_check_vertices(Workspace& ws, hipStream_t s, MeshView m, int* err);
void launch_quadrics(hipStream_t s, MeshView m, double* Q, int* err);
// mesh_done (batches, may be null): edges of finished meshes get no key
// cost_target > 0: edges costing more get the largest key (never chosen);
// prefilter: so do edges failing the local checks of R7 (link condition,
// degenerate or flipped generated triangles; m needs this round's stars)
void launch_cost_keys(Workspace& ws, hipStream_t s, MeshView m, const double* Q, double w_e, double w_s,
                      const uint8_t* demote, const uint8_t* mesh_done, uint64_t* key, int* err,
                      double cost_target = 0.0, bool prefilter = false, bool lex = false);
// float64 key mode, after launch_cost_keys(lex): each keyed edge's key becomes
// (rank in the order of (float64 cost, edge id)) << 32 | edge id
void launch_rank_keys(Workspace& ws, hipStream_t s, MeshView m, uint64_t* key);
// the vertex minima of key gathered into vmin (one thread per vertex over its
// stored star, no atomics), then the selection and its compaction
// sel_clear: the selection flags ("sel", 3 nf bytes) are known to be zero
// (a compaction given them cleared them), else they are cleared first
void launch_select(Workspace& ws, hipStream_t s, MeshView m, const uint64_t* key, uint64_t* vmin, int* cand,
                   int* ncand, bool sel_clear = false);
// the selection again after the candidates dlist[0..*nd) (*nd <= bound) got
// the largest key on both half-edges: into cand / ncand the same candidates as
// a full launch_select, from the flags and vertex minima of the selection
// before (m needs the stored stars of this round)
void launch_reselect(Workspace& ws, hipStream_t s, MeshView m, const uint64_t* key, uint64_t* vmin, const int* dlist,
                     const int* nd, int bound, int* cand, int* ncand);
void launch_local_check(hipStream_t s, MeshView m, const double* Q, double w_e, double w_s, const int* cand,
                        const int* ncand, int cand_bound, const uint64_t* key, uint8_t* reason, double* vbar,
                        uint64_t* ckey, int* err, int* hist);
void launch_cap(Workspace& ws, hipStream_t s, const int* ncand, int nc_host, const uint64_t* ckey, uint8_t* reason,
                int64_t need);
void launch_face_boxes(hipStream_t s, MeshView m, float* box);
// ovl[f] = ovl_new[f] for the alive faces of committed collapses
void launch_ovl_commit(hipStream_t s, int nf, const int* owner, const uint8_t* falive, const int* undone,
                       const int* ovl_new, int* ovl, const int* gate = nullptr);
// one launch for a round's check state: falive = 1, owner = -1 and (box not
// null) the float32 box of every face, undone[0..ncand) = 0, valive (not
// null) = 1
void launch_round_prep(hipStream_t s, MeshView m, float* box, uint8_t* falive, int* owner, int ncand, int* undone,
                       uint8_t* valive);
// falive[0..nf) = 1, owner[0..nf) = -1, undone[0..ncand) = 0
void launch_check_reset(hipStream_t s, int nf, uint8_t* falive, int* owner, int ncand, int* undone);
void launch_apply(hipStream_t s, MeshView m, const int* cand, const int* ncand, int cand_bound, const uint8_t* reason,
                  const double* vbar, double* oldpos, int* owner, uint8_t* falive, float* box);
void launch_undo(hipStream_t s, MeshView m, const int* cand, const int* ncand, int cand_bound, const int* undone,
                 int iter, const double* oldpos, uint8_t* falive);
// faces changed by an applied collapse (iter = 0) or restored by the undo of
// check iteration iter (iter >= 1), ascending
// (in the order of `order` when given: a permutation of the faces)
void launch_face_list(Workspace& ws, hipStream_t s, int nf, const int* owner, const uint8_t* falive,
                      const int* undone, int iter, const int* order, int* list, int* count);
// Kernels given a gate do nothing when *gate != 0.  The gate is set when the
// check pass must be read back before the round can end: a collapse was
// undone, more candidate pairs than cap, an error bit, or (npass given) no
// collapse passed the local checks.  The commit kernel evaluates it from these
// counters (GateIn) and stores it for the kernels after it.
struct GateIn {
  const int* nundo = nullptr;
  const int* ncandp = nullptr;
  const int* err = nullptr;
  const int* npass = nullptr;
  int cap = 0;
  int* flag = nullptr;  // null: no gate to evaluate
};

void launch_commit(hipStream_t s, MeshView m, const int* cand, const int* ncand, int cand_bound, uint8_t* reason,
                   const int* undone, uint8_t* valive, GateIn gin = GateIn{});
// flags of rejected edges; hist (may be null) += histogram of the reasons
void launch_flags(hipStream_t s, MeshView m, const int* cand, const int* ncand, int cand_bound, const uint8_t* reason,
                  int* hist = nullptr, const int* gate = nullptr);
void launch_flags_or(hipStream_t s, uint8_t* dst, const uint8_t* src, int64_t n);
void launch_reason_hist(hipStream_t s, const int* ncand, int cand_bound, const uint8_t* reason, int* hist);
// order (optional): a leaf order of the source faces, whose surviving faces go
// to order_out (new ids, the count to *nord); order_out must not be order;
// sel (optional): 3 bytes per surviving face set to zero (the next round's
// selection flags)
// (f_off, v_off, nmesh): a batch's per-mesh offsets, updated to the compacted numbering
void launch_compact(Workspace& ws, hipStream_t s, MeshView src, MeshView dst, const uint8_t* falive,
                    const uint8_t* valive, int* nf_new, int* nv_new, int* err, const int* gate = nullptr,
                    const int* order = nullptr, int* order_out = nullptr, int* nord = nullptr, int* f_off = nullptr,
                    int* v_off = nullptr, int nmesh = 0, uint8_t* sel = nullptr);
void launch_clear_u8(hipStream_t s, uint8_t* p, int64_t n, const int* gate);

// ------------------------------------------------------------ LBVH
// 4-wide node: the boxes of its four children as structure of arrays (child
// c: lo (lx[c], ly[c], lz[c]), hi (hx[c], hy[c], hz[c]); an absent child has
// lo = +inf, hi = -inf and meets nothing).  128 bytes, two cache lines.
struct __align__(16) BvhNode {
  float4 lx, ly, lz, hx, hy, hz;
  int4 leaf;  // at the last internal level: face of each child leaf (-1 = none)
  int4 pad;
};

// balanced implicit 4-ary tree over 4^D Hilbert-sorted leaf slots: internal
// node k at level l (0 <= l < D, (4^l - 1)/3 <= k < (4^(l+1) - 1)/3) has
// children 4k+1 .. 4k+4; slot j of the leaves is child j % 4 of the node at
// position j / 4 of level D - 1.  Nodes whose leaves all lie past n are never
// entered (their parents record them as empty) and are not written.
constexpr int LEAF_CHANGED = 1 << 30;  // leaf record flags: the face was changed this round,
constexpr int LEAF_DEAD = 1 << 29;     // the face was deleted by a tentative collapse
constexpr int LEAF_ID = LEAF_DEAD - 1;
constexpr int BVH_DMAX = 14;  // 4^14 leaf slots; stack entries pack a node index below 2^27
struct Bvh {
  BvhNode* nodes;
  const int* sorted;  // faces in Hilbert order (leaf j holds sorted[j])
  int n;              // faces
  int D;              // internal levels
};

// ------------------------------------------------------------ batches
// per-mesh tallies of one round: candidates, passing candidates, commits,
// final reasons, deepest undo iteration (arrays of nmesh, cleared by caller)
void launch_mesh_tally(hipStream_t s, const int* cand, const int* ncand, int bound, const int* fmesh,
                       const uint8_t* reason_local, const uint8_t* reason_final, const int* undone, int* ncand_m,
                       int* npass_m, int* commits_m, int* hist_m, int* undo_m, const int* gate = nullptr);
// exact-target cap per mesh: keep the need[m] smallest keys among the passing
// candidates of mesh m
void launch_cap_batch(Workspace& ws, hipStream_t s, const int* ncand, int nc_host, const int* cand,
                      const int* fmesh, const uint64_t* ckey, uint8_t* reason, const int* need_m,
                      const int* ncand_m, int nmesh);
// clear the flags of meshes that committed a collapse this round
void launch_flags_clear_batch(hipStream_t s, MeshView m, const int* commits_m, const int* gate = nullptr);
// F + v_off[mesh]: local to global vertex ids (local ids outside [0, nv of
// the mesh) raise PAMO_EBIT_INDEX); fmesh/vmesh from the offsets (nmesh + 1 each)
void launch_batch_ids(hipStream_t s, const int* f_off, const int* v_off, int nmesh, int nf, int nv, int* F,
                      int* fmesh, int* vmesh, int* err);
// new per-mesh offsets after a compaction (rank of the first survivor)
void launch_batch_offsets(Workspace& ws, hipStream_t s, const uint8_t* alive, int n, int* off, int nmesh);
// write mesh m's output at out offsets: faces with local vertex ids
void launch_batch_output(hipStream_t s, MeshView m, const int* f_off, const int* v_off, const int* f_out_off,
                         const int* v_out_off, int nmesh, double* V_out, int* F_out);

// build over the face boxes box[f] (6 floats, lo then hi), all nf faces.
// `order` (may be null): a permutation of the faces to use as leaf order
// instead of sorting by the Hilbert index of the box centres (any order gives
// a correct tree; a near-Hilbert order gives a good one).
// fmesh (batches, may be null): sort by (mesh, Hilbert index of the unshifted box)
// node records the build writes for nf leaves (sum over heights h >= 1 of
// ceil(nf / 4^h), 128 bytes each)
inline int64_t bvh_nodes_written(int64_t nf) {
  int64_t total = 0;
  for (int64_t c = nf; c > 1;) {
    c = (c + 3) / 4;
    total += c;
  }
  return total;
}
// owner, falive (may be null): leaves of faces with owner[f] >= 0 carry
// LEAF_CHANGED, those with falive[f] == 0 LEAF_DEAD in their record (face id =
// record & LEAF_ID); the flags hold for the first check pass of the round
// reserve the BVH builder's buffers for up to nf leaves (mesh_codes: the
// batch form's 64-bit (mesh, Hilbert) codes too); its sort is reserved by
// prim_reserve
void bvh_reserve(Workspace& ws, int64_t nf, bool mesh_codes);
Bvh build_bvh(Workspace& ws, hipStream_t s, const float* box, int nf, const int* order, const int* fmesh = nullptr,
              int nmesh = 1, const int* owner = nullptr, const uint8_t* falive = nullptr);
// new leaf order after a stable compaction: keep the alive faces of `order`
// in sequence, renamed by fmap
void launch_remap_order(Workspace& ws, hipStream_t s, const int* order, int nf_old, const uint8_t* falive,
                        const int* fmap, int* out, int* count);

enum QueryMode { QUERY_CHANGED = 0, QUERY_RESTORED = 1, QUERY_ALL_PAIRS = 2 };

struct QueryArgs {
  const double* V;
  const int* F;
  const uint8_t* falive;  // may be null: all alive
  const int* owner;       // QUERY_CHANGED / QUERY_RESTORED
  int* undone;            // marks, CAS 0 -> iter
  int iter;
  int* nundo;             // newly undone collapses
  int2* defer;            // pairs the float filter could not decide
  int* ndefer;
  int defer_cap;
  int2* pairs;            // QUERY_ALL_PAIRS output (t < u)
  int* npairs;
  int64_t pairs_cap;
  int2* cand;             // candidate pairs collected by the traversal
  int* ncand;
  int cand_cap;
  const int* fmesh;       // batches: mesh of each face (query boxes are shifted like the tree's)
  int* ovl_cnt;           // when set: per query face, the alive faces sharing no vertex whose boxes meet it
  int* err;
};

// queries: qlist[0..*nq) (device count), nq_bound >= *nq for the grid size.
// Traversal collects candidate pairs into a.cand (count a.ncand, which may
// exceed a.cand_cap: then the caller grows the buffer and repeats).
// `packet`: queries per traversal packet (1, 2, 4, 8, 16, 32 or 64), or
// `coop` > 1: lanes sharing one query (2, 4, 8 or 16; trees up to 2^24 leaves)
void launch_query(hipStream_t s, const Bvh& bvh, QueryMode mode, const int* qlist, const int* nq, int nq_bound,
                  const QueryArgs& a, int packet, int coop);
// the pair predicate on the collected pairs (grid sized for about pairs_est
// pairs; the kernel strides over the device count)
void launch_pairs(hipStream_t s, QueryMode mode, const QueryArgs& a, int64_t pairs_est);
// settle the deferred pairs exactly
void launch_resolve(hipStream_t s, QueryMode mode, const QueryArgs& a);

}  // namespace pamo
