// Host side of the library: contexts, the round driver of
// ParallelSimplification (PaMO Sec. 5) and the C ABI of include/pamo.h.
//
// One round on the device (all kernels on the context stream):
//   quadrics -> cost/keys -> vertex minima -> selection + compaction      [read ncand]
//   local checks -> reason histogram                                      [read passing]
//   (exact-target cap) -> face boxes -> tentative apply -> LBVH build
//   changed-face list -> query -> exact resolve of deferred pairs         [read undone]
//   { undo -> restored-face list -> query -> resolve }*                   [read undone]
//   commit -> flags -> stable compaction                                  [read nf, nv]
// The host reads back a handful of counters per round to size launches and
// to decide the loop; everything else stays on the GPU.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "internal.hpp"
#include "learn.hpp"
#include "project.hpp"
#include "remesh.hpp"
#include "round.hpp"
#include "exact_dev.hpp"

using namespace pamo;

// Phases timed on request with HIP events on the context stream.  Each
// carries its algorithmic byte count: the bytes the phase must move at
// minimum (every input element read once, every output written once).
enum Phase {
  PH_QUADRICS, PH_COST, PH_SELECT, PH_LOCAL, PH_CAP, PH_BOXES, PH_APPLY, PH_BVH, PH_FACELIST, PH_QUERY,
  PH_PAIRS, PH_RESOLVE, PH_UNDO, PH_COMMIT, PH_FLAGS, PH_COMPACT, PH_LEARN, PH_COUNT
};
static const char* const PH_NAME[PH_COUNT] = {
    "quadrics", "cost_keys", "select", "local_check", "cap", "face_boxes", "apply", "bvh_build",
    "face_list", "query", "pairs", "resolve", "undo", "commit", "flags", "compact", "learn"};

struct Prof {
  uint32_t mask = 0;
  struct Acc {
    int64_t launches = 0;
    double ms = 0, bytes = 0;
  } acc[PH_COUNT];
  struct Pending {
    int ph;
    hipEvent_t a, b;
    double bytes;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
};

// defaults of the tuning knobs (chosen by the autotuner on the 1.31M-face
// workload; none of them changes a result)
constexpr int PAMO_DEFAULT_PACKET = 1;
constexpr int PAMO_DEFAULT_COOP = 8;
constexpr int PAMO_DEFAULT_COOP_BELOW = 65536;
constexpr int PAMO_DEFAULT_RESORT = 1 << 30;  // never: the first round's Hilbert order, carried along

struct pamo_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  pamo_options opt{};
  std::string err;
  Workspace ws;
  int* hcnt = nullptr;  // pinned mirror of the device counters
  int* dcnt = nullptr;
  int* hbt = nullptr;   // pinned mirror of the per-mesh tallies of a batch
  size_t hbt_n = 0;
  Prof prof;
  MlpDev* mlp = nullptr;  // the learned proposal's network (device), when set
  void* scratch = nullptr;  // device address of this device's static scratch (pamo_simplify_noalloc)
};

namespace {

enum {
  C_NCAND = 0,   // candidates selected this round
  C_NQ = 1,      // queries of the current pass
  C_NUNDO = 2,   // collapses newly undone by the current check pass
  C_NDEFER = 3,  // pairs deferred to the exact predicate
  C_NCANDP = 4,  // candidate pairs collected by one query pass
  C_NPAIRS = 5,  // intersecting pairs (whole-mesh test)
  C_NF = 6,      // faces / vertices after compaction
  C_NV = 7,
  C_HIST = 8,    // 8 entries: reason histogram after the local checks
  C_HIST2 = 16,  // 8 entries: final reason histogram
  C_ERR = 24,    // error bits
  C_NORD = 25,   // length of the remapped leaf order
  C_NDEMOTE = 26,  // candidates set aside by the network this round
  C_NROWS = 27,    // training rows logged this round
  C_GATE = 28,     // the round's check must be read back before it can end
  C_COUNT = 32
};

struct Fail {
  pamo_status code;
  std::string msg;
};

void fail(pamo_status code, const std::string& msg) { throw Fail{code, msg}; }

// Scratch of pamo_simplify_noalloc: a file-scope device array that every GPU
// the library runs on holds until the process ends.  In host code the array's
// name is not a device address: each device's copy is found once, with that
// device current, by hipGetSymbolAddress (scratch_address, from pamo_create),
// and only that address is used afterwards.
static __device__ __align__(256) unsigned char scratch[PAMO_NOALLOC_SCRATCH_BYTES];

constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[SCRATCH_DEVICES] = {};

// device address of `scratch` on `device`, which must be current
void* scratch_address(int device) {
  if (device < 0 || device >= SCRATCH_DEVICES) fail(PAMO_ERR_ARG, "device index outside [0, 64)");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* p = nullptr;
    PAMO_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(PAMO_ERR_HIP, "no device address for the static scratch");
    g_scratch_addr[device] = p;
  }
  return g_scratch_addr[device];
}

hipEvent_t ev_get(pamo_ctx* c) {
  if (!c->prof.pool.empty()) {
    hipEvent_t e = c->prof.pool.back();
    c->prof.pool.pop_back();
    return e;
  }
  hipEvent_t e;
  PAMO_HIP(hipEventCreate(&e));
  return e;
}

// fold finished timings into the accumulators (the stream is synchronised)
void prof_resolve(pamo_ctx* c) {
  for (auto& p : c->prof.pending) {
    float ms = 0;
    PAMO_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    auto& a = c->prof.acc[p.ph];
    a.launches++;
    a.ms += ms;
    a.bytes += p.bytes;
    c->prof.pool.push_back(p.a);
    c->prof.pool.push_back(p.b);
  }
  c->prof.pending.clear();
}

struct Scope {
  pamo_ctx* c;
  int ph;
  double bytes;
  hipEvent_t a = nullptr;
  Scope(pamo_ctx* c_, int ph_, double bytes_) : c(c_), ph(ph_), bytes(bytes_) {
    if (c->prof.mask & (1u << ph)) {
      a = ev_get(c);
      PAMO_HIP(hipEventRecord(a, c->stream));
    }
  }
  ~Scope() {
    if (!a) return;
    hipEvent_t b = nullptr;
    if (hipEventCreate(&b) == hipSuccess && hipEventRecord(b, c->stream) == hipSuccess)
      c->prof.pending.push_back({ph, a, b, bytes});
  }
};
#define PAMO_CAT2(a, b) a##b
#define PAMO_CAT(a, b) PAMO_CAT2(a, b)
#define TIMED(ph, bytes) Scope PAMO_CAT(scope_, __LINE__)(c, ph, (double)(bytes))

// add algorithmic bytes to a phase after the fact (counts known only later)
void prof_bytes(pamo_ctx* c, int ph, double bytes) {
  if (c->prof.mask & (1u << ph)) c->prof.acc[ph].bytes += bytes;
}

const int* readback(pamo_ctx* c) {
  PAMO_HIP(hipMemcpyAsync(c->hcnt, c->dcnt, C_COUNT * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  PAMO_HIP(hipStreamSynchronize(c->stream));
  if (!c->prof.pending.empty()) prof_resolve(c);
  return c->hcnt;
}

void check_err_bits(int e) {
  if (!e) return;
  if (e & PAMO_EBIT_INDEX) fail(PAMO_ERR_ARG, "a face refers to a vertex index outside [0, nv)");
  if (e & PAMO_EBIT_DEGENERATE) fail(PAMO_ERR_DEGENERATE, "a face repeats a vertex");
  if (e & PAMO_EBIT_EDGE) fail(PAMO_ERR_NONMANIFOLD, "an edge does not have exactly two faces (open or non-manifold mesh)");
  if (e & PAMO_EBIT_ORIENT) fail(PAMO_ERR_NONMANIFOLD, "the two faces of an edge are inconsistently oriented");
  if (e & PAMO_EBIT_VERTEX) fail(PAMO_ERR_NONMANIFOLD, "an unused vertex or a non-manifold vertex");
  if (e & PAMO_EBIT_RING) fail(PAMO_ERR_NONMANIFOLD, "a vertex star is corrupt or too long");
  if (e & PAMO_EBIT_STACK) fail(PAMO_ERR_CAPACITY, "BVH traversal stack overflow");
  if (e & PAMO_EBIT_DEFER) fail(PAMO_ERR_CAPACITY, "too many pairs for the exact predicate");
  if (e & PAMO_EBIT_TILES) fail(PAMO_ERR_CAPACITY, "a triangle's band reaches too many tiles of the grid");
  fail(PAMO_ERR_HIP, "unknown device error");
}

MeshView mesh_bufs(Workspace& w, const char* tag, int64_t nv, int64_t nf) {
  std::string t(tag);
  MeshView m;
  m.V = w.get<double>(t + ".V", 3 * nv);
  m.F = w.get<int>(t + ".F", 3 * nf);
  m.twin = w.get<int>(t + ".twin", 3 * nf);
  m.vh = w.get<int>(t + ".vh", nv);
  m.flags = w.get<uint8_t>(t + ".flags", 3 * nf);
  m.nv = (int)nv;
  m.nf = (int)nf;
  return m;
}

void check_sizes(int64_t nv, int64_t nf) {
  if (nv < 4 || nf < 4) fail(PAMO_ERR_ARG, "a closed mesh needs at least 4 vertices and 4 faces");
  if (nf > (int64_t)(INT32_MAX / 3) - 1 || nv > INT32_MAX - 1) fail(PAMO_ERR_ARG, "mesh too large for int32 ids");
}

// copy the caller's mesh into `m`, build twins / leaving half-edges, validate
void load_mesh(pamo_ctx* c, MeshView m, const double* V, const int32_t* F, const uint8_t* flags) {
  hipStream_t s = c->stream;
  PAMO_HIP(hipMemcpyAsync(m.V, V, 3 * (size_t)m.nv * sizeof(double), hipMemcpyDeviceToDevice, s));
  PAMO_HIP(hipMemcpyAsync(m.F, F, 3 * (size_t)m.nf * sizeof(int), hipMemcpyDeviceToDevice, s));
  if (flags)
    PAMO_HIP(hipMemcpyAsync(m.flags, flags, 3 * (size_t)m.nf, hipMemcpyDeviceToDevice, s));
  else
    fill_u8(s, m.flags, 3 * (int64_t)m.nf, 0);
  fill_i32(s, c->dcnt, C_COUNT, 0);
  launch_adjacency(c->ws, s, m, c->dcnt + C_ERR);
  const int* h = readback(c);
  check_err_bits(h[C_ERR]);
  launch_check_vertices(c->ws, s, m, c->dcnt + C_ERR);
  h = readback(c);
  check_err_bits(h[C_ERR]);
}

struct RoundBufs {
  double* Q;
  uint64_t* key;
  uint64_t* vmin;
  int* cand;
  uint8_t* reason;
  double* vbar;
  double* oldpos;
  uint64_t* ckey;
  int* owner;
  int* undone;
  uint8_t* falive;
  uint8_t* valive;
  float* box;
  int* qlist;
  int2* defer;
  int defer_cap;
  int* morder;   // leaf order carried between rounds (see Driver)
  int* morder2;  // the next order while a round is not yet confirmed
  int* vstar;    // per-vertex star faces, star sizes and neighbour boxes (written by the quadrics kernel)
  int* vdeg;
  double* vbox;
  int* ovl_new;  // learned proposal: overlap counts measured this round (null when not tracked)
  float* X;      // learned proposal: features of this round's candidates (null when unused)
  int* dlist;    // learned proposal: the edges the network set aside this round
  bool sel_clear;  // the selection flags are zero (the last compaction cleared them)
};

// one query pass (traversal + pair predicate + exact resolve); grows the
// candidate-pair buffer and repeats when it overflowed (marks are idempotent)
// lanes per query for a pass of about nq_est queries (0: one lane per query)
int coop_lanes(const pamo_ctx* c, int64_t nq_est) {
  const int below = c->opt.coop_below > 0 ? c->opt.coop_below : PAMO_DEFAULT_COOP_BELOW;
  if (c->opt.query_coop == 1 || nq_est >= below) return 0;
  return c->opt.query_coop > 1 ? c->opt.query_coop : PAMO_DEFAULT_COOP;
}

// the kernels of one query pass: traversal, pair predicate, exact resolve.
// nq_est: about how many queries the pass has (sizes grids, picks the walk)
void query_launch(pamo_ctx* c, const Bvh& bvh, QueryMode mode, const int* qlist, int* nq_dev, int bound,
                  int64_t nq_est, QueryArgs& qa, double bytes) {
  hipStream_t s = c->stream;
  const int packet = c->opt.query_packet > 0 ? c->opt.query_packet : PAMO_DEFAULT_PACKET;
  const int coop = coop_lanes(c, nq_est);
  if (qa.ovl_cnt) fill_i32(s, qa.ovl_cnt, bvh.n, 0);  // counted afresh by every attempt
  {
    TIMED(PH_QUERY, bytes);
    launch_query(s, bvh, mode, qlist, nq_dev, bound, qa, packet, coop);
  }
  {
    TIMED(PH_PAIRS, 0);  // bytes added once the pair count is known
    launch_pairs(s, mode, qa, 16 * nq_est);
  }
  {
    TIMED(PH_RESOLVE, 0);
    launch_resolve(s, mode, qa);
  }
}

// given the counters h read back after a pass: when the candidate-pair buffer
// overflowed, grow it and repeat the pass (marks are idempotent, and the
// undone count stands), until one fits
const int* query_settle(pamo_ctx* c, const Bvh& bvh, QueryMode mode, const int* qlist, int* nq_dev, int bound,
                        int64_t nq_est, QueryArgs& qa, double bytes, double vbytes, const int* h) {
  for (;;) {
    check_err_bits(h[C_ERR]);
    const int np = std::min(h[C_NCANDP], qa.cand_cap);
    prof_bytes(c, PH_PAIRS, 8.0 * np + vbytes);
    if (h[C_NCANDP] <= qa.cand_cap) return h;
    int64_t cap = (int64_t)h[C_NCANDP] + h[C_NCANDP] / 4 + 1024;
    if (cap > INT32_MAX / 2) fail(PAMO_ERR_CAPACITY, "too many candidate pairs");
    qa.cand = c->ws.get<int2>("q.pairs", cap);
    qa.cand_cap = (int)cap;
    fill_i32(c->stream, c->dcnt + C_NDEFER, 3, 0);  // repeat: marks and the undone count stand
    query_launch(c, bvh, mode, qlist, nq_dev, bound, nq_est, qa, bytes);
    h = readback(c);
  }
}

// one whole query pass, read back
const int* query_pass(pamo_ctx* c, const Bvh& bvh, QueryMode mode, const int* qlist, int* nq_dev, int bound,
                      int64_t nq_est, QueryArgs& qa, double bytes, double vbytes) {
  fill_i32(c->stream, c->dcnt + C_NUNDO, 4, 0);  // undone, deferred, collected, intersecting
  query_launch(c, bvh, mode, qlist, nq_dev, bound, nq_est, qa, bytes);
  return query_settle(c, bvh, mode, qlist, nq_dev, bound, nq_est, qa, bytes, vbytes, readback(c));
}

// initial capacity of the candidate-pair buffer of a query pass (grown and
// the pass repeated when it overflows)
int64_t pair_capacity(const pamo_options& o, int64_t nf) {
  if (o.pair_capacity > 0) return o.pair_capacity;
  return std::min<int64_t>(std::max<int64_t>(1 << 20, 16 * nf), INT32_MAX / 2);
}

void init_pair_buffer(pamo_ctx* c, QueryArgs& qa, int64_t nf) {
  int64_t cap = pair_capacity(c->opt, nf);
  qa.cand = c->ws.get<int2>("q.pairs", cap);
  qa.cand_cap = (int)std::min<int64_t>(cap, INT32_MAX / 2);
  qa.ncand = c->dcnt + C_NCANDP;
}

RoundBufs round_bufs(Workspace& w, int64_t nv, int64_t nf) {
  RoundBufs b;
  int64_t nh = 3 * nf;
  b.Q = w.get<double>("r.Q", 10 * nv);
  b.key = w.get<uint64_t>("r.key", nh);
  b.vmin = w.get<uint64_t>("r.vmin", nv);
  b.cand = w.get<int>("r.cand", nh);
  b.reason = w.get<uint8_t>("r.reason", nh);
  b.vbar = w.get<double>("r.vbar", 3 * nh);
  b.oldpos = w.get<double>("r.oldpos", 3 * nh);
  b.ckey = w.get<uint64_t>("r.ckey", nh);
  b.owner = w.get<int>("r.owner", nf);
  b.undone = w.get<int>("r.undone", nh);
  b.falive = w.get<uint8_t>("r.falive", nf);
  b.valive = w.get<uint8_t>("r.valive", nv);
  b.box = w.get<float>("r.box", 6 * nf);
  b.qlist = w.get<int>("r.qlist", nf);
  b.defer_cap = (int)std::max<int64_t>(1 << 16, nf);
  b.defer = w.get<int2>("r.defer", b.defer_cap);
  b.morder = w.get<int>("r.morder", nf);
  b.morder2 = w.get<int>("r.morder2", nf);
  b.vstar = w.get<int>("r.vstar", VSTAR * nv);
  b.vdeg = w.get<int>("r.vdeg", nv);
  b.vbox = w.get<double>("r.vbox", 6 * nv);
  b.ovl_new = nullptr;
  b.X = nullptr;
  b.dlist = nullptr;
  b.sel_clear = false;
  return b;
}

// Which optional parts of the path a call can reach.
struct Parts {
  int nmesh = 1;         // > 1: the batched form (per-mesh ids and tallies)
  bool learned = false;  // overlap counts, features and the set-aside list of the learned proposal
  bool collect = false;  // training-row logging (pamo_collect)
};

// Reserve every buffer a mesh entry point can request, at its largest size for
// a mesh (or batch) of nv vertices and nf faces: later requests of the call
// then fit their blocks, so an arena is carved once and the size query
// (counting mode) is the exact total.  Sizes are the round-0 sizes (meshes
// only shrink); candidates of a round are at most nf / 2 + 1 (their rings are
// disjoint).
void reserve_mesh(Workspace& w, int64_t nv, int64_t nf, const pamo_options& o, const Parts& p) {
  const int64_t bound = nf / 2 + 1;
  mesh_bufs(w, "mA", nv, nf);
  mesh_bufs(w, "mB", nv, nf);
  if (p.nmesh > 1) {
    w.get<int>("mA.fmesh", nf);
    w.get<int>("mA.vmesh", nv);
    w.get<int>("mB.fmesh", nf);
    w.get<int>("mB.vmesh", nv);
    w.get<int>("bt.dev", 15 * (int64_t)p.nmesh + 2);
    w.get<int>("bt.need", p.nmesh);
    w.get<uint8_t>("bt.done", p.nmesh);
    w.get<uint8_t>("bt.use", p.nmesh);
  }
  round_bufs(w, nv, nf);
  if (o.prefilter) {  // the pre-filter's edges left to the exact flip test
    w.get<int>("ck.late", 3 * nf / 2 + 1);
    w.get<int>("ck.nlate", 1);
  }
  w.get<int2>("q.pairs", pair_capacity(o, nf));
  w.get<int>("ord.copy", nf);
  w.get<float>("w.box", 6 * nf);
  w.get<int2>("w.defer", std::max<int64_t>(1 << 16, nf));
  w.get<int2>("w.pairs", 1);
  if (p.learned || p.collect) {
    w.get<int>("mA.ovl", nf);
    w.get<int>("mB.ovl", nf);
    w.get<int>("r.ovl_new", nf);
    w.get<float>("r.X", bound * (int64_t)LEARN_NFEAT);
    w.get<int>("r.dlist", bound);
  }
  if (p.collect) {
    w.get<double>("col.V", 3 * nv);
    w.get<int>("col.F", 3 * nf);
    learn_reserve(w, bound);
  }
  bvh_reserve(w, nf, p.nmesh > 1);
  round_reserve(w, nv, nf, bound, p.nmesh, o.key_mode != 0);
  prim_reserve(w, 3 * nf, nf, 3 * nf, 2 * nf + nv);
}

// the reservation of a mesh entry point (arena mode only: owned buffers grow
// on demand)
void reserve(pamo_ctx* c, int64_t nv, int64_t nf, const Parts& p) {
  if (c->ws.arena) reserve_mesh(c->ws, nv, nf, c->opt, p);
}

struct RoundResult {
  int ncand = 0, npass = 0, chosen = 0, undone = 0, commits = 0, iters = 0, deferred = 0;
  int hist[8] = {0};
  const int* leaf_order = nullptr;  // the BVH leaf order used this round (null: no BVH built)
  int demoted = 0;     // learned proposal: candidates set aside
  bool retry = false;  // learned proposal: set-aside round committed nothing; rerun it plain
};

// The learned proposal's share of a run: setting candidates aside with the
// network, keeping the per-face overlap counts its features read, and logging
// training rows (features and outcome of each candidate the checks decided).
struct LearnRun {
  bool learned = false;
  bool active = false;  // consult the network this round (the previous round's checks rejected something)
  bool track = false;
  float* X = nullptr;  // logging: rows [cap][32] and labels [cap] (device)
  uint8_t* y = nullptr;
  int64_t cap = 0, n = 0;
  int64_t demoted = 0, fallbacks = 0;
};

// Leaf order of the BVH carried across rounds: sorting by Hilbert index every
// round is replaced by the previous order, stably remapped through the
// compaction, with a fresh sort every `resort` rounds.  Any order gives a
// correct tree; this only affects speed.
struct OrderState {
  bool valid = false;
  int age = 0;
  int resort = 4;
  int chosen_est = 0;  // collapses applied by the previous round (sizes the next query when not read back)
};

// Local checks of the candidates (link, degeneracy, flip) and the histogram
// of their outcome.  `bound` >= *ncand_dev sizes the grid (selected edges
// have disjoint rings of at least two faces, so nf / 2 always bounds them).
void local_checks(pamo_ctx* c, MeshView m, const RoundBufs& b, const int* cand, const int* ncand_dev, int bound,
                  uint8_t* reason, double* vbar) {
  hipStream_t s = c->stream;
  int* cnt = c->dcnt;
  {
    TIMED(PH_LOCAL, 0);  // bytes are added once the candidate count is known
    launch_local_check(s, m, b.Q, c->opt.w_e, c->opt.w_s, cand, ncand_dev, bound, b.key, reason, vbar, b.ckey,
                       cnt + C_ERR, cnt + C_HIST);  // C_HIST zeroed with the round's counters
  }
}

// exact face target of a single mesh: keep the `need` smallest keys
void cap_single(pamo_ctx* c, const RoundBufs& b, const int* ncand_dev, uint8_t* reason, int64_t teff, int nf,
                RoundResult& R) {
  int64_t need = (nf - teff) / 2;
  R.chosen = R.npass;
  if (R.npass > need) {
    TIMED(PH_CAP, 8 * 16.0 * R.ncand);
    launch_cap(c->ws, c->stream, ncand_dev, R.ncand, b.ckey, reason, need);
    R.chosen = (int)need;
  }
}

// A check/undo fixed point between the launch of its first query pass and
// its resolution.
struct CheckRun {
  Bvh bvh{};
  QueryArgs qa{};
  double qbytes = 0, pbytes = 0;
};

// Tentative apply of the R.chosen collapses with reason 0 on `m`, the BVH,
// the list of changed faces and the first query pass, all enqueued, nothing
// read back.  Returns false when nothing was applied (no pass launched).
// `order`: BVH leaf order to reuse, or null to sort.
bool check_launch(pamo_ctx* c, MeshView m, const RoundBufs& b, const int* cand, const int* ncand_dev, int ncand,
                  uint8_t* reason, double* vbar, const RoundResult& R, const int* order, int nmesh, int* ovl_new,
                  CheckRun& K) {
  hipStream_t s = c->stream;
  int* cnt = c->dcnt;
  const double nf = m.nf, nv = m.nv;
  {
    TIMED(PH_BOXES, 36 * nf + 24 * nv);
    launch_round_prep(s, m, R.chosen > 0 ? b.box : nullptr, b.falive, b.owner, ncand, b.undone, b.valive);
  }
  if (R.chosen == 0) return false;
  {
    TIMED(PH_APPLY, 900.0 * R.chosen);
    launch_apply(s, m, cand, ncand_dev, ncand, reason, vbar, b.oldpos, b.owner, b.falive, b.box);
  }
  {
    TIMED(PH_BVH, 24 * nf + 128.0 * bvh_nodes_written(m.nf));
    K.bvh = build_bvh(c->ws, s, b.box, m.nf, order, m.fmesh, nmesh, b.owner, b.falive);
  }
  {
    TIMED(PH_FACELIST, 8 * nf);
    launch_face_list(c->ws, s, m.nf, b.owner, b.falive, b.undone, 0, K.bvh.sorted, b.qlist, cnt + C_NQ);
  }
  QueryArgs& qa = K.qa;
  qa = QueryArgs{};
  qa.V = m.V;
  qa.F = m.F;
  qa.falive = b.falive;
  qa.owner = b.owner;
  qa.undone = b.undone;
  qa.iter = 1;
  qa.nundo = cnt + C_NUNDO;
  qa.defer = b.defer;
  qa.ndefer = cnt + C_NDEFER;
  qa.defer_cap = b.defer_cap;
  qa.fmesh = m.fmesh;
  qa.err = cnt + C_ERR;
  init_pair_buffer(c, qa, m.nf);
  K.qbytes = 128.0 * bvh_nodes_written(m.nf) + 17 * nf + 24 * nv;  // tree + faces + alive/owner + vertices
  K.pbytes = 17 * nf + 24 * nv;  // pairs: faces, alive/owner, vertices (+ 8 per pair)
  qa.ovl_cnt = ovl_new;          // overlap counts of the changed faces on the tentative mesh
  // the counters of the pass (undone, deferred, collected, intersecting) are
  // still zero from the start of the round: every caller clears them there
  query_launch(c, K.bvh, QUERY_CHANGED, b.qlist, cnt + C_NQ, m.nf, 10ll * R.chosen, qa, K.qbytes);
  return true;
}

// The rest of the fixed point, given the counters h read back after the first
// pass: a pass that overflowed is repeated, then every undone collapse is
// restored and the faces it restored are checked again until nothing is
// undone.  `m` is left with the surviving collapses applied.
void check_resolve(pamo_ctx* c, MeshView m, const RoundBufs& b, const int* cand, const int* ncand_dev, int ncand,
                   RoundResult& R, CheckRun& K, const int* h) {
  hipStream_t s = c->stream;
  int* cnt = c->dcnt;
  const double nf = m.nf;
  QueryArgs& qa = K.qa;
  h = query_settle(c, K.bvh, QUERY_CHANGED, b.qlist, cnt + C_NQ, m.nf, 10ll * R.chosen, qa, K.qbytes, K.pbytes, h);
  qa.ovl_cnt = nullptr;
  int newly = h[C_NUNDO];
  R.deferred += h[C_NDEFER];
  while (newly > 0) {
    R.undone += newly;
    R.iters++;
    {
      TIMED(PH_UNDO, 200.0 * newly);
      launch_undo(s, m, cand, ncand_dev, ncand, b.undone, R.iters, b.oldpos, b.falive);
    }
    {
      TIMED(PH_FACELIST, 8 * nf);
      launch_face_list(c->ws, s, m.nf, b.owner, b.falive, b.undone, R.iters, K.bvh.sorted, b.qlist, cnt + C_NQ);
    }
    qa.iter = R.iters + 1;
    h = query_pass(c, K.bvh, QUERY_RESTORED, b.qlist, cnt + C_NQ, m.nf, 10ll * newly, qa, K.qbytes, K.pbytes);
    newly = h[C_NUNDO];
    R.deferred += h[C_NDEFER];
  }
  R.commits = R.chosen - R.undone;
  R.leaf_order = K.bvh.sorted;
}

// Tentative apply of the R.chosen collapses with reason 0 and the check/undo
// fixed point on `m` (modified: undone collapses restored, applied ones left
// applied).  undone[c] != 0 marks collapses undone by the loop (reason not yet
// set to 3).  `order`: BVH leaf order to reuse, or null to sort.
void check_and_undo(pamo_ctx* c, MeshView m, const RoundBufs& b, const int* cand, const int* ncand_dev, int ncand,
                    uint8_t* reason, double* vbar, RoundResult& R, const int* order, int nmesh = 1,
                    int* ovl_new = nullptr) {
  CheckRun K;
  if (!check_launch(c, m, b, cand, ncand_dev, ncand, reason, vbar, R, order, nmesh, ovl_new, K)) return;
  check_resolve(c, m, b, cand, ncand_dev, ncand, R, K, readback(c));
}

void add_stats(pamo_stats* st, const RoundResult& R) {
  st->rounds++;
  st->candidates += R.ncand;
  st->commits += R.commits;
  st->rej_link += R.hist[1];
  st->rej_flip += R.hist[2];
  st->rej_isect += R.hist[3];
  st->capped += R.hist[4];
  st->undo_hist[std::min(R.iters, 4)]++;
  st->deferred_pairs += R.deferred;
}

// The end of a round once the check is settled (or speculatively, gated):
// commit the surviving collapses, next round's invalid flags (this round's
// rejections, plus the old flags when nothing was collapsed, Sec. 5.3),
// compaction into `alt`, and the BVH leaf order remapped into `order_out`.
void round_tail(pamo_ctx* c, MeshView& cur, MeshView& alt, const RoundBufs& b, const RoundResult& R, LearnRun* L,
                const GateIn& gin, int* order_out) {
  const int* gate = gin.flag;
  hipStream_t s = c->stream;
  int* cnt = c->dcnt;
  const double nf = cur.nf, nv = cur.nv;
  const bool logging = L && L->X;
  if (R.chosen > 0) {
    TIMED(PH_COMMIT, 100.0 * R.chosen);
    launch_commit(s, cur, b.cand, cnt + C_NCAND, R.ncand, b.reason, b.undone, b.valive, gin);  // evaluates the gate
  }
  if (L && L->track && R.chosen > 0)
    launch_ovl_commit(s, cur.nf, b.owner, b.falive, b.undone, b.ovl_new, cur.ovl, gate);
  if (logging && L->n < L->cap) {
    TIMED(PH_LEARN, 0);
    launch_log_rows(c->ws, s, cnt + C_NCAND, R.ncand, b.reason, b.X, L->X + L->n * LEARN_NFEAT, L->y + L->n,
                    L->cap - L->n, cnt + C_NROWS);
  }
  {
    TIMED(PH_FLAGS, 3 * nf + 10.0 * R.ncand);
    if (R.commits > 0) launch_clear_u8(s, cur.flags, 3 * (int64_t)cur.nf, gate);
    launch_flags(s, cur, b.cand, cnt + C_NCAND, R.ncand, b.reason, cnt + C_HIST2, gate);
  }
  if (R.commits > 0) {
    TIMED(PH_COMPACT, 72 * nf + 66 * nv);
    // the leaf order follows the compaction (through a copy when it would be
    // remapped in place)
    const int* src = R.leaf_order;
    if (src && src == order_out) {
      int* tmp = c->ws.get<int>("ord.copy", cur.nf);
      PAMO_HIP(hipMemcpyAsync(tmp, src, (size_t)cur.nf * sizeof(int), hipMemcpyDeviceToDevice, s));
      src = tmp;
    }
    launch_compact(c->ws, s, cur, alt, b.falive, b.valive, cnt + C_NF, cnt + C_NV, cnt + C_ERR, gate, src, order_out,
                   cnt + C_NORD, nullptr, nullptr, 0, c->ws.get<uint8_t>("sel", 3 * (int64_t)cur.nf));
  } else if (R.leaf_order && R.leaf_order != order_out) {
    PAMO_HIP(hipMemcpyAsync(order_out, R.leaf_order, (size_t)cur.nf * sizeof(int), hipMemcpyDeviceToDevice, s));
  }
}

// given the counters read back after round_tail: reasons, logged rows, and the
// compacted mesh becomes current
RoundResult round_end(pamo_ctx* c, MeshView& cur, MeshView& alt, RoundResult& R, LearnRun* L, const int* h) {
  check_err_bits(h[C_ERR]);
  for (int i = 0; i < 8; i++) R.hist[i] = h[C_HIST2 + i];
  if (L && L->X) L->n += std::min<int64_t>(h[C_NROWS], L->cap - L->n);
  if (R.commits > 0) {
    alt.nf = h[C_NF];
    alt.nv = h[C_NV];
    std::swap(cur, alt);
  }
  return R;
}

// One full round on `cur`.  When collapses are committed, the compacted mesh
// lands in `alt` and the two views are swapped.
RoundResult run_round(pamo_ctx* c, MeshView& cur, MeshView& alt, RoundBufs& b, int64_t teff, OrderState& os,
                      LearnRun* L = nullptr) {
  hipStream_t s = c->stream;
  int* cnt = c->dcnt;
  RoundResult R;
  fill_i32(s, cnt, C_COUNT, 0);
  const double nf = cur.nf, nv = cur.nv;
  const bool learned = L && L->learned && L->active;
  const bool logging = L && L->X;
  cur.vstar = b.vstar;
  cur.vdeg = b.vdeg;
  cur.vbox = b.vbox;
  {
    TIMED(PH_QUADRICS, 224 * nv + 24 * nf);
    launch_quadrics(s, cur, b.Q, cnt + C_ERR);
  }
  {
    TIMED(PH_COST, 220 * nv + 51 * nf);
    launch_cost_keys(c->ws, s, cur, b.Q, c->opt.w_e, c->opt.w_s, nullptr, nullptr, b.key, cnt + C_ERR, c->opt.cost_target,
                     c->opt.prefilter != 0, c->opt.key_mode != 0);
  }
  {
    TIMED(PH_SELECT, 84 * nv + 45 * nf);
    if (c->opt.key_mode) launch_rank_keys(c->ws, s, cur, b.key);
    launch_select(c->ws, s, cur, b.key, b.vmin, b.cand, cnt + C_NCAND, b.sel_clear);
    b.sel_clear = false;
  }
  const int bound = cur.nf / 2 + 1;
  if (learned || logging) {
    TIMED(PH_LEARN, 0);
    launch_features(s, cur, b.key, b.cand, cnt + C_NCAND, bound, cur.ovl, b.X, cnt + C_ERR);
    if (learned) {
      launch_mlp(s, b.X, cnt + C_NCAND, bound, c->mlp, nullptr, b.cand, cur.twin, b.key, cnt + C_NDEMOTE, nullptr,
                 nullptr, nullptr, b.dlist);
      launch_reselect(c->ws, s, cur, b.key, b.vmin, b.dlist, cnt + C_NDEMOTE, bound, b.cand,
                      cnt + C_NCAND);  // without the set-aside edges
    }
  }
  local_checks(c, cur, b, b.cand, cnt + C_NCAND, bound, b.reason, b.vbar);
  int* ovl_new = L && L->track ? b.ovl_new : nullptr;
  // no training rows logged (the network may be consulted, overlap counts kept)
  const bool plain = !logging;
  // The exact-target cap cannot bind while nf >= 2 teff: selected edges have
  // disjoint rings of at least four faces, so at most nf / 4 pass, and
  // nf / 4 <= (nf - teff) / 2.  The plain method then goes on without reading
  // the candidate counts back: grids take the bound, the device the counts.
  const bool blind = plain && cur.nf >= 2 * teff;
  const int* h = nullptr;
  if (blind) {
    R.ncand = bound;
    // an estimate until the end of the round (it sizes the query grids): the
    // previous round's count, or about one collapse per 32 faces at first
    R.chosen = R.npass = std::max(1, os.chosen_est > 0 ? os.chosen_est : cur.nf / 32);
  } else {
    h = readback(c);
    check_err_bits(h[C_ERR]);
    R.ncand = h[C_NCAND];
    R.npass = h[C_HIST + 0];
    R.demoted = h[C_NDEMOTE];
    prof_bytes(c, PH_LOCAL, 780.0 * R.ncand);
    if (R.ncand == 0) {  // nothing selectable: a round without collapses
      R.retry = learned && R.demoted > 0;
      return R;
    }
  }
  const bool reuse = os.valid && os.age < os.resort;
  if (!blind) cap_single(c, b, cnt + C_NCAND, b.reason, teff, cur.nf, R);
  // Speculative end of round (no training rows logged, something to apply):
  // the round's tail is enqueued right behind the first query
  // pass, its kernels gated on the device.  When that pass undid nothing,
  // fitted its pair buffer and set no error bit, the round ends with this one
  // read-back; otherwise the tail did nothing and the check is finished the
  // usual way.
  if (plain && R.chosen > 0) {
    CheckRun K;
    check_launch(c, cur, b, b.cand, cnt + C_NCAND, R.ncand, b.reason, b.vbar, R, reuse ? b.morder : nullptr, 1,
                 ovl_new, K);
    GateIn gin;
    gin.nundo = cnt + C_NUNDO;
    gin.ncandp = cnt + C_NCANDP;
    gin.err = cnt + C_ERR;
    gin.npass = blind ? cnt + C_HIST : nullptr;
    gin.cap = K.qa.cand_cap;
    gin.flag = cnt + C_GATE;
    R.commits = R.chosen;  // if nothing is undone
    R.leaf_order = K.bvh.sorted;
    round_tail(c, cur, alt, b, R, L, gin, b.morder2);
    h = readback(c);
    if (blind) {
      R.ncand = h[C_NCAND];
      R.chosen = R.npass = h[C_HIST + 0];
      R.demoted = h[C_NDEMOTE];
      prof_bytes(c, PH_LOCAL, 780.0 * R.ncand);
    }
    os.chosen_est = R.chosen;
    if (!h[C_GATE]) {
      prof_bytes(c, PH_PAIRS, 8.0 * h[C_NCANDP] + K.pbytes);
      R.commits = R.chosen;
      R.deferred += h[C_NDEFER];
      os.age = reuse ? os.age + 1 : 1;
      os.valid = true;
      std::swap(b.morder, b.morder2);
      b.sel_clear = true;  // the speculative compaction ran
      return round_end(c, cur, alt, R, L, h);
    }
    R.commits = 0;
    R.leaf_order = nullptr;
    check_resolve(c, cur, b, b.cand, cnt + C_NCAND, R.ncand, R, K, h);
  } else {
    check_and_undo(c, cur, b, b.cand, cnt + C_NCAND, R.ncand, b.reason, b.vbar, R, reuse ? b.morder : nullptr, 1,
                   ovl_new);
  }
  if (learned && R.demoted > 0 && R.commits == 0) {
    // everything was undone, so the mesh is as the round found it
    R.retry = true;
    return R;
  }
  if (R.leaf_order) {
    os.age = reuse ? os.age + 1 : 1;
    os.valid = true;
  }
  round_tail(c, cur, alt, b, R, L, GateIn{}, b.morder);
  b.sel_clear = R.commits > 0;  // a compaction ran
  return round_end(c, cur, alt, R, L, readback(c));
}

// a learned round that set candidates aside and committed nothing runs again
// without the network
RoundResult run_round_learned(pamo_ctx* c, MeshView& cur, MeshView& alt, RoundBufs& b, int64_t teff,
                              OrderState& os, LearnRun* L) {
  RoundResult R = run_round(c, cur, alt, b, teff, os, L);
  if (!L) return R;
  L->demoted += R.demoted;
  if (R.retry) {
    L->fallbacks++;
    LearnRun plain = *L;
    plain.learned = false;
    R = run_round(c, cur, alt, b, teff, os, &plain);
    L->n = plain.n;
  }
  return R;
}

__global__ void k_iota(int* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i;
}

__global__ void k_check_index(const int* F, int64_t n3, int nv, int* err) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n3 && (F[i] < 0 || F[i] >= nv)) atomicOr(err, PAMO_EBIT_INDEX);
}

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t > 0 ? (n + t - 1) / t : 1); }

// all intersecting pairs of the mesh m; returns their number
int64_t whole_mesh_pairs(pamo_ctx* c, MeshView m, int2* pairs, int64_t cap, int nmesh = 1, int* ovl = nullptr) {
  hipStream_t s = c->stream;
  int* cnt = c->dcnt;
  float* box = c->ws.get<float>("w.box", 6 * (int64_t)m.nf);

  int defer_cap = (int)std::max<int64_t>(1 << 16, m.nf);
  int2* defer = c->ws.get<int2>("w.defer", defer_cap);
  fill_i32(s, cnt, C_COUNT, 0);
  fill_i32(s, cnt + C_NQ, 1, m.nf);
  launch_face_boxes(s, m, box);
  Bvh bvh = build_bvh(c->ws, s, box, m.nf, nullptr, m.fmesh, nmesh);
  const int* ql = bvh.sorted;  // every face, in Hilbert order
  QueryArgs qa{};
  qa.V = m.V;
  qa.F = m.F;
  qa.fmesh = m.fmesh;
  qa.defer = defer;
  qa.ndefer = cnt + C_NDEFER;
  qa.defer_cap = defer_cap;
  qa.pairs = pairs;
  qa.npairs = cnt + C_NPAIRS;
  qa.pairs_cap = cap;
  qa.err = cnt + C_ERR;
  qa.ovl_cnt = ovl;
  init_pair_buffer(c, qa, m.nf);
  const int* h = query_pass(c, bvh, QUERY_ALL_PAIRS, ql, cnt + C_NQ, m.nf, m.nf, qa, 0, 0);
  return h[C_NPAIRS];
}

__global__ void k_tri_pairs(const double* P, const int* ip, const double* Q, const int* iq, int64_t n, uint8_t* out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  P3 a[3], b[3];
  int ia[3], ib[3];
  for (int k = 0; k < 3; k++) {
    a[k] = P3{P[9 * i + 3 * k], P[9 * i + 3 * k + 1], P[9 * i + 3 * k + 2]};
    b[k] = P3{Q[9 * i + 3 * k], Q[9 * i + 3 * k + 1], Q[9 * i + 3 * k + 2]};
    ia[k] = ip[3 * i + k];
    ib[k] = iq[3 * i + k];
  }
  out[i] = (uint8_t)tri_pair<true>(a, ia, b, ib);
}

template <class Fn>
pamo_status guarded(pamo_ctx* c, Fn&& fn) {
  if (!c) return PAMO_ERR_ARG;
  try {
    PAMO_HIP(hipSetDevice(c->device));
    c->err.clear();
    c->ws.begin_call();
    c->dcnt = c->ws.get<int>("ctx.cnt", C_COUNT);  // first in an arena
    return fn();
  } catch (const Fail& f) {
    c->err = f.msg;
    return f.code;
  } catch (const WorkspaceFull& e) {
    c->err = e.what();
    return PAMO_ERR_CAPACITY;
  } catch (const HipError& e) {
    c->err = e.what();
    return PAMO_ERR_HIP;
  } catch (const std::exception& e) {
    c->err = e.what();
    return PAMO_ERR_HIP;
  } catch (...) {
    c->err = "unknown failure";
    return PAMO_ERR_HIP;
  }
}

int32_t read_count(pamo_ctx* c, const int32_t* dev) {
  int32_t v = 0;
  PAMO_HIP(hipMemcpyAsync(&v, dev, sizeof(v), hipMemcpyDeviceToHost, c->stream));
  PAMO_HIP(hipStreamSynchronize(c->stream));
  return v;
}


// ------------------------------------------------------------------ batches
// A batch is the disjoint union of its meshes in one set of arrays, with the
// mesh of every face and vertex (fmesh, vmesh) carried through compaction.
// Every launch of a round covers all meshes; nothing in a round crosses from
// one mesh to another (rings are mesh-local, the BVH pair filter compares
// mesh ids), so each mesh follows exactly the rounds it would follow alone.
// A mesh that has stopped keeps no candidate (its edges get no key) and
// therefore stays as it is.  Stable compaction keeps the meshes contiguous and
// in order, so per-mesh offsets are the only bookkeeping.

// per-mesh tallies on the device, one block so that one copy reads them all
struct Batch {
  int n = 0;
  int* dev = nullptr;      // [T_COUNT]
  int* need = nullptr;     // [n] collapses still needed (0 for stopped meshes)
  uint8_t* done = nullptr; // [n]
  uint8_t* use = nullptr;  // [n] consult the network for this mesh this round
  int ncand_m() const { return 0; }
  int npass_m() const { return n; }
  int commits_m() const { return 2 * n; }
  int undo_m() const { return 3 * n; }
  int hist_m() const { return 4 * n; }
  int demote_m() const { return 12 * n; }
  int f_off() const { return 13 * n; }
  int v_off() const { return 14 * n + 1; }
  int total() const { return 15 * n + 2; }
  int* d(int o) const { return dev + o; }
};

Batch batch_bufs(pamo_ctx* c, int n) {
  Batch B;
  B.n = n;
  B.dev = c->ws.get<int>("bt.dev", B.total());
  B.need = c->ws.get<int>("bt.need", n);
  B.done = c->ws.get<uint8_t>("bt.done", n);
  B.use = c->ws.get<uint8_t>("bt.use", n);
  size_t want = (size_t)B.total() + n + 2 * ((n + 3) / 4);
  if (c->hbt_n < want) {
    if (c->hbt) PAMO_HIP(hipHostFree(c->hbt));
    c->hbt = nullptr;
    c->hbt_n = 0;
    PAMO_HIP(hipHostMalloc((void**)&c->hbt, want * sizeof(int)));
    c->hbt_n = want;
  }
  return B;
}

// host staging of the per-round uploads, behind the tally mirror
int* host_need(pamo_ctx* c, const Batch& B) { return c->hbt + B.total(); }
uint8_t* host_done(pamo_ctx* c, const Batch& B) { return (uint8_t*)(c->hbt + B.total() + B.n); }
uint8_t* host_use(pamo_ctx* c, const Batch& B) { return (uint8_t*)(c->hbt + B.total() + B.n + (B.n + 3) / 4); }

// counters and tallies in one synchronisation
const int* readback_batch(pamo_ctx* c, const Batch& B) {
  PAMO_HIP(hipMemcpyAsync(c->hcnt, c->dcnt, C_COUNT * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  PAMO_HIP(hipMemcpyAsync(c->hbt, B.dev, B.total() * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  PAMO_HIP(hipStreamSynchronize(c->stream));
  if (!c->prof.pending.empty()) prof_resolve(c);
  return c->hcnt;
}

struct MeshRun {
  int64_t teff = 0;
  int streak = 0;
  bool settled = false;  // cost target: a round selected nothing, the mesh is done
  bool active = false;
  bool rejected = false;  // the mesh's previous round had check rejections
  pamo_stats st{};
};

// The end of a batch round (gated like round_tail): commit, per-mesh tallies
// of the outcome, overlap counts, flags (cleared only in meshes that
// committed), compaction with the per-mesh offsets and the leaf order.
void batch_tail(pamo_ctx* c, MeshView& cur, MeshView& alt, const RoundBufs& b, const Batch& B, const RoundResult& R,
                bool track, bool learned, const GateIn& gin, int* order_out) {
  hipStream_t s = c->stream;
  int* cnt = c->dcnt;
  const int n = B.n;
  const double nf = cur.nf, nv = cur.nv;
  const int* gate = gin.flag;
  if (R.chosen > 0) {
    TIMED(PH_COMMIT, 100.0 * R.chosen);
    launch_commit(s, cur, b.cand, cnt + C_NCAND, R.ncand, b.reason, b.undone, b.valive, gin);  // evaluates the gate
  }
  launch_mesh_tally(s, b.cand, cnt + C_NCAND, R.ncand, cur.fmesh, nullptr, b.reason, b.undone, nullptr, nullptr,
                    B.d(B.commits_m()), B.d(B.hist_m()), B.d(B.undo_m()), gate);
  if (track && R.chosen > 0) launch_ovl_commit(s, cur.nf, b.owner, b.falive, b.undone, b.ovl_new, cur.ovl, gate);
  if (learned)  // meshes whose round runs again keep their flags
    launch_mark_retry(s, b.cand, cnt + C_NCAND, R.ncand, cur.fmesh, B.d(B.demote_m()), B.d(B.commits_m()), b.reason,
                      gate);
  {
    TIMED(PH_FLAGS, 3 * nf + 10.0 * R.ncand);
    if (R.commits > 0) launch_flags_clear_batch(s, cur, B.d(B.commits_m()), gate);
    launch_flags(s, cur, b.cand, cnt + C_NCAND, R.ncand, b.reason, cnt + C_HIST2, gate);
  }
  if (R.commits > 0) {
    TIMED(PH_COMPACT, 72 * nf + 66 * nv);
    const int* src = R.leaf_order;
    if (src && src == order_out) {  // remapping in place: go through a copy
      int* tmp = c->ws.get<int>("ord.copy", cur.nf);
      PAMO_HIP(hipMemcpyAsync(tmp, src, (size_t)cur.nf * sizeof(int), hipMemcpyDeviceToDevice, s));
      src = tmp;
    }
    launch_compact(c->ws, s, cur, alt, b.falive, b.valive, cnt + C_NF, cnt + C_NV, cnt + C_ERR, gate, src, order_out,
                   cnt + C_NORD, B.d(B.f_off()), B.d(B.v_off()), n, c->ws.get<uint8_t>("sel", 3 * (int64_t)cur.nf));
  } else if (R.leaf_order && R.leaf_order != order_out) {
    PAMO_HIP(hipMemcpyAsync(order_out, R.leaf_order, (size_t)cur.nf * sizeof(int), hipMemcpyDeviceToDevice, s));
  }
}

// One round over every mesh of the batch (the single-mesh round of run_round
// with per-mesh targets, tallies, flag clearing and offsets).
RoundResult run_round_batch(pamo_ctx* c, MeshView& cur, MeshView& alt, RoundBufs& b, const Batch& B,
                            std::vector<MeshRun>& mr, OrderState& os, bool learned = false, bool track = false) {
  hipStream_t s = c->stream;
  int* cnt = c->dcnt;
  const int n = B.n;
  RoundResult R;
  fill_i32(s, cnt, C_COUNT, 0);
  fill_i32(s, B.dev, B.f_off(), 0);  // tallies; the offsets stay
  int* hneed = host_need(c, B);
  uint8_t* hdone = host_done(c, B);
  for (int m = 0; m < n; m++) {
    int64_t nfm = c->hbt[B.f_off() + m + 1] - c->hbt[B.f_off() + m];
    hneed[m] = mr[m].active ? (int)((nfm - mr[m].teff) / 2) : 0;
    hdone[m] = mr[m].active ? 0 : 1;
  }
  PAMO_HIP(hipMemcpyAsync(B.need, hneed, n * sizeof(int), hipMemcpyHostToDevice, s));
  PAMO_HIP(hipMemcpyAsync(B.done, hdone, n, hipMemcpyHostToDevice, s));
  if (learned) {
    uint8_t* huse = host_use(c, B);
    bool any = false;
    for (int m = 0; m < n; m++) {
      huse[m] = mr[m].active && mr[m].rejected;
      any |= huse[m] != 0;
    }
    learned = any;
    if (any) PAMO_HIP(hipMemcpyAsync(B.use, huse, n, hipMemcpyHostToDevice, s));
  }
  const double nf = cur.nf, nv = cur.nv;
  cur.vstar = b.vstar;
  cur.vdeg = b.vdeg;
  cur.vbox = b.vbox;
  {
    TIMED(PH_QUADRICS, 224 * nv + 24 * nf);
    launch_quadrics(s, cur, b.Q, cnt + C_ERR);
  }
  {
    TIMED(PH_COST, 220 * nv + 51 * nf);
    launch_cost_keys(c->ws, s, cur, b.Q, c->opt.w_e, c->opt.w_s, nullptr, B.done, b.key, cnt + C_ERR, c->opt.cost_target,
                     c->opt.prefilter != 0, c->opt.key_mode != 0);
  }
  {
    TIMED(PH_SELECT, 84 * nv + 45 * nf);
    if (c->opt.key_mode) launch_rank_keys(c->ws, s, cur, b.key);
    launch_select(c->ws, s, cur, b.key, b.vmin, b.cand, cnt + C_NCAND, b.sel_clear);
    b.sel_clear = false;
  }
  const int bound = cur.nf / 2 + 1;
  if (learned) {
    TIMED(PH_LEARN, 0);
    launch_features(s, cur, b.key, b.cand, cnt + C_NCAND, bound, cur.ovl, b.X, cnt + C_ERR, cur.fmesh, B.use);
    launch_mlp(s, b.X, cnt + C_NCAND, bound, c->mlp, nullptr, b.cand, cur.twin, b.key, cnt + C_NDEMOTE, cur.fmesh,
               B.d(B.demote_m()), B.use, b.dlist);
    launch_reselect(c->ws, s, cur, b.key, b.vmin, b.dlist, cnt + C_NDEMOTE, bound, b.cand, cnt + C_NCAND);
  }
  local_checks(c, cur, b, b.cand, cnt + C_NCAND, bound, b.reason, b.vbar);
  launch_mesh_tally(s, b.cand, cnt + C_NCAND, bound, cur.fmesh, b.reason, nullptr, nullptr, B.d(B.ncand_m()),
                    B.d(B.npass_m()), nullptr, nullptr, nullptr);
  // as in run_round: no mesh's exact-target cap can bind while every active
  // mesh has nf_m >= 2 teff_m, so the plain batch then goes on without
  // reading the candidate counts back
  bool blind = true;
  for (int m = 0; m < n && blind; m++) {
    const int64_t nfm = c->hbt[B.f_off() + m + 1] - c->hbt[B.f_off() + m];
    if (mr[m].active && nfm < 2 * mr[m].teff) blind = false;
  }
  const int* h = nullptr;
  if (blind) {
    R.ncand = bound;
    R.chosen = R.npass = std::max(1, os.chosen_est > 0 ? os.chosen_est : cur.nf / 32);  // estimate (sizes grids)
  } else {
    h = readback_batch(c, B);
    check_err_bits(h[C_ERR]);
    R.ncand = h[C_NCAND];
    R.npass = h[C_HIST + 0];
    prof_bytes(c, PH_LOCAL, 780.0 * R.ncand);
    if (R.ncand == 0) return R;
    bool capped = false;
    R.chosen = 0;
    for (int m = 0; m < n; m++) {
      int np = c->hbt[B.npass_m() + m];
      if (np > hneed[m]) capped = true;
      R.chosen += std::min(np, hneed[m]);
    }
    if (capped) {
      TIMED(PH_CAP, 8 * 16.0 * R.ncand);
      launch_cap_batch(c->ws, s, cnt + C_NCAND, R.ncand, b.cand, cur.fmesh, b.ckey, b.reason, B.need,
                       B.d(B.ncand_m()), n);
    }
  }
  const bool reuse = os.valid && os.age < os.resort;
  int* ovl_new = track ? b.ovl_new : nullptr;
  if (R.chosen > 0) {
    // speculative end of round, gated on the device (see run_round)
    CheckRun K;
    check_launch(c, cur, b, b.cand, cnt + C_NCAND, R.ncand, b.reason, b.vbar, R, reuse ? b.morder : nullptr, n,
                 ovl_new, K);
    GateIn gin;
    gin.nundo = cnt + C_NUNDO;
    gin.ncandp = cnt + C_NCANDP;
    gin.err = cnt + C_ERR;
    gin.npass = blind ? cnt + C_HIST : nullptr;
    gin.cap = K.qa.cand_cap;
    gin.flag = cnt + C_GATE;
    R.commits = R.chosen;
    R.leaf_order = K.bvh.sorted;
    batch_tail(c, cur, alt, b, B, R, track, learned, gin, b.morder2);
    h = readback_batch(c, B);
    if (blind) {
      R.ncand = h[C_NCAND];
      R.chosen = R.npass = h[C_HIST + 0];
      prof_bytes(c, PH_LOCAL, 780.0 * R.ncand);
    }
    os.chosen_est = R.chosen;
    if (!h[C_GATE]) {
      prof_bytes(c, PH_PAIRS, 8.0 * h[C_NCANDP] + K.pbytes);
      R.commits = R.chosen;
      R.deferred += h[C_NDEFER];
      os.age = reuse ? os.age + 1 : 1;
      os.valid = true;
      std::swap(b.morder, b.morder2);
      b.sel_clear = true;  // the speculative compaction ran
      return round_end(c, cur, alt, R, nullptr, h);
    }
    R.commits = 0;
    R.leaf_order = nullptr;
    check_resolve(c, cur, b, b.cand, cnt + C_NCAND, R.ncand, R, K, h);
  } else {
    check_and_undo(c, cur, b, b.cand, cnt + C_NCAND, R.ncand, b.reason, b.vbar, R, reuse ? b.morder : nullptr, n,
                   ovl_new);
  }
  if (R.leaf_order) {
    os.age = reuse ? os.age + 1 : 1;
    os.valid = true;
  }
  batch_tail(c, cur, alt, b, B, R, track, learned, GateIn{}, b.morder);
  b.sel_clear = R.commits > 0;  // a compaction ran
  return round_end(c, cur, alt, R, nullptr, readback_batch(c, B));
}

// the whole method on one mesh (plain, learned, or plain with row logging)
pamo_status simplify_run(pamo_ctx* c, const double* V, int64_t nv, const int32_t* F, int64_t nf, int64_t target_faces,
                         double* V_out, int64_t* nv_out, int32_t* F_out, int64_t* nf_out, pamo_stats* stats,
                         LearnRun* L) {
  check_sizes(nv, nf);
  if (target_faces < 0) fail(PAMO_ERR_ARG, "negative target");
  if (L->learned && !c->mlp) fail(PAMO_ERR_ARG, "the learned proposal needs a network (pamo_set_mlp)");
  if (L->learned && c->opt.key_mode)
    fail(PAMO_ERR_ARG, "the learned proposal's features read the float32 cost from the key (key_mode 0)");
  hipStream_t s = c->stream;
  Parts parts;
  parts.learned = L->track;
  parts.collect = L->X != nullptr;
  reserve(c, nv, nf, parts);
  MeshView cur = mesh_bufs(c->ws, "mA", nv, nf);
  MeshView alt = mesh_bufs(c->ws, "mB", nv, nf);
  load_mesh(c, cur, V, F, nullptr);
  if (c->opt.validate_input) {
    int2* dummy = c->ws.get<int2>("w.pairs", 1);
    if (whole_mesh_pairs(c, cur, dummy, 0) > 0) fail(PAMO_ERR_SELF_INTERSECTING, "the input intersects itself");
  }
  RoundBufs b = round_bufs(c->ws, nv, nf);
  if (L->track) {
    cur.ovl = c->ws.get<int>("mA.ovl", nf);
    alt.ovl = c->ws.get<int>("mB.ovl", nf);
    b.ovl_new = c->ws.get<int>("r.ovl_new", nf);
    b.X = c->ws.get<float>("r.X", (nf / 2 + 1) * (int64_t)LEARN_NFEAT);
    b.dlist = c->ws.get<int>("r.dlist", nf / 2 + 1);
    int2* dummy = c->ws.get<int2>("w.pairs", 1);
    whole_mesh_pairs(c, cur, dummy, 0, 1, cur.ovl);
  }
  pamo_stats st;
  memset(&st, 0, sizeof(st));
  int64_t teff = target_faces - target_faces % 2;
  int streak = 0;
  pamo_status status = PAMO_OK;
  OrderState os;
  os.resort = c->opt.resort_every > 0 ? c->opt.resort_every : PAMO_DEFAULT_RESORT;
  for (;;) {
    if (cur.nf <= teff) break;
    if (streak >= c->opt.tolerance) {
      status = PAMO_TARGET_UNREACHED;
      break;
    }
    if (c->opt.max_rounds >= 0 && st.rounds >= c->opt.max_rounds) break;
    RoundResult R = run_round_learned(c, cur, alt, b, teff, os, L);
    add_stats(&st, R);
    streak = R.commits == 0 ? streak + 1 : 0;
    // with a cost target, a round that selects nothing ends the run: every
    // edge is flagged or above the target, and the next round would be the same
    if (c->opt.cost_target > 0 && R.ncand == 0) break;
    L->active = R.hist[1] + R.hist[2] + R.hist[3] > 0;  // the network has something to predict
  }
  PAMO_HIP(hipMemcpyAsync(V_out, cur.V, 3 * (size_t)cur.nv * sizeof(double), hipMemcpyDeviceToDevice, s));
  PAMO_HIP(hipMemcpyAsync(F_out, cur.F, 3 * (size_t)cur.nf * sizeof(int), hipMemcpyDeviceToDevice, s));
  PAMO_HIP(hipStreamSynchronize(s));
  *nv_out = cur.nv;
  *nf_out = cur.nf;
  st.faces_out = cur.nf;
  st.verts_out = cur.nv;
  st.status = status;
  st.demoted = L->demoted;
  st.fallbacks = L->fallbacks;
  if (stats) *stats = st;
  return status;
}

}  // namespace

// ============================================================== C ABI
extern "C" {

void pamo_default_options(pamo_options* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->w_e = 0.001;
  o->w_s = 0.005;
  o->tolerance = 4;
  o->max_rounds = -1;
  o->validate_input = 0;
}

pamo_status pamo_create(pamo_ctx** out, int device, void* hip_stream, const pamo_options* opt) {
  if (!out) return PAMO_ERR_ARG;
  *out = nullptr;
  pamo_ctx* c = new (std::nothrow) pamo_ctx();
  if (!c) return PAMO_ERR_ARG;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  pamo_default_options(&c->opt);
  if (opt) c->opt = *opt;
  if (hipSetDevice(device) != hipSuccess || hipHostMalloc((void**)&c->hcnt, C_COUNT * sizeof(int)) != hipSuccess) {
    if (c->hcnt) (void)hipHostFree(c->hcnt);
    delete c;
    return PAMO_ERR_HIP;
  }
  try {
    c->scratch = scratch_address(device);  // once per device, with the device current
  } catch (...) {
    (void)hipHostFree(c->hcnt);
    delete c;
    return PAMO_ERR_HIP;
  }
  *out = c;
  return PAMO_OK;
}

void pamo_destroy(pamo_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto& p : c->prof.pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : c->prof.pool) (void)hipEventDestroy(e);
  c->ws.release();
  if (c->hcnt) (void)hipHostFree(c->hcnt);
  if (c->hbt) (void)hipHostFree(c->hbt);
  if (c->mlp) (void)hipFree(c->mlp);
  delete c;
}

pamo_status pamo_set_options(pamo_ctx* c, const pamo_options* opt) {
  if (!c || !opt) return PAMO_ERR_ARG;
  if (opt->tolerance < 1) return PAMO_ERR_ARG;
  if (opt->resort_every < 0) return PAMO_ERR_ARG;
  int qp = opt->query_packet;
  if (qp != 0 && qp != 1 && qp != 2 && qp != 4 && qp != 8 && qp != 16 && qp != 32 && qp != 64) return PAMO_ERR_ARG;
  int qc = opt->query_coop;
  if (qc != 0 && qc != 1 && qc != 2 && qc != 4 && qc != 8 && qc != 16) return PAMO_ERR_ARG;
  if (opt->coop_below < 0) return PAMO_ERR_ARG;
  if (opt->pair_capacity < 0 || opt->pair_capacity > INT32_MAX / 2) return PAMO_ERR_ARG;
  c->opt = *opt;
  return PAMO_OK;
}

const char* pamo_last_error(const pamo_ctx* c) { return c ? c->err.c_str() : "null context"; }

int64_t pamo_workspace_held(const pamo_ctx* c) { return c && !c->ws.arena ? (int64_t)c->ws.total : 0; }

size_t pamo_workspace_bytes(int64_t nv, int64_t nf, const pamo_options* opt) {
  if (nv < 4 || nf < 4 || nf > (int64_t)(INT32_MAX / 3) - 1 || nv > INT32_MAX - 1) return 0;
  pamo_options o;
  pamo_default_options(&o);
  if (opt) o = *opt;
  try {
    Workspace w;
    w.counting = true;
    w.get<int>("ctx.cnt", C_COUNT);
    Parts p;
    p.nmesh = PAMO_MAX_MESHES;
    p.learned = true;
    p.collect = true;
    reserve_mesh(w, nv, nf, o, p);
    return w.total;
  } catch (...) {
    return 0;
  }
}

pamo_status pamo_set_workspace(pamo_ctx* c, void* dev, size_t bytes) {
  return guarded(c, [&]() -> pamo_status {
    if (dev && ((uintptr_t)dev % 256 != 0)) fail(PAMO_ERR_ARG, "workspace must be 256-byte aligned");
    if (dev && bytes < 4096) fail(PAMO_ERR_ARG, "workspace smaller than 4 KiB");
    PAMO_HIP(hipStreamSynchronize(c->stream));  // owned buffers may still be in use
    c->ws.set_arena(dev, bytes);
    c->dcnt = nullptr;  // taken again at the start of every call
    return PAMO_OK;
  });
}

pamo_status pamo_quadrics(pamo_ctx* c, const double* V, int64_t nv, const int32_t* F, int64_t nf, double* Q) {
  return guarded(c, [&]() -> pamo_status {
    if (!V || !F || !Q) fail(PAMO_ERR_ARG, "null pointer");
    check_sizes(nv, nf);
    reserve(c, nv, nf, Parts{});
    MeshView A = mesh_bufs(c->ws, "mA", nv, nf);
    load_mesh(c, A, V, F, nullptr);
    launch_quadrics(c->stream, A, Q, c->dcnt + C_ERR);
    check_err_bits(readback(c)[C_ERR]);
    return PAMO_OK;
  });
}

pamo_status pamo_select(pamo_ctx* c, const double* V, int64_t nv, const int32_t* F, int64_t nf,
                        const uint8_t* flags, const uint8_t* demote, uint64_t* keys, int32_t* cand, int32_t* ncand) {
  return guarded(c, [&]() -> pamo_status {
    if (!V || !F || !cand || !ncand) fail(PAMO_ERR_ARG, "null pointer");
    check_sizes(nv, nf);
    reserve(c, nv, nf, Parts{});
    MeshView A = mesh_bufs(c->ws, "mA", nv, nf);
    load_mesh(c, A, V, F, flags);
    RoundBufs b = round_bufs(c->ws, nv, nf);
    uint64_t* key = keys ? keys : b.key;
    launch_quadrics(c->stream, A, b.Q, c->dcnt + C_ERR);
    launch_cost_keys(c->ws, c->stream, A, b.Q, c->opt.w_e, c->opt.w_s, demote, nullptr, key, c->dcnt + C_ERR,
                     c->opt.cost_target, c->opt.prefilter != 0, c->opt.key_mode != 0);
    if (c->opt.key_mode) launch_rank_keys(c->ws, c->stream, A, key);
    launch_select(c->ws, c->stream, A, key, b.vmin, cand, ncand);
    check_err_bits(readback(c)[C_ERR]);
    return PAMO_OK;
  });
}

pamo_status pamo_check(pamo_ctx* c, const double* V, int64_t nv, const int32_t* F, int64_t nf,
                       const uint8_t* flags, int64_t target_faces, const int32_t* cand, const int32_t* ncand,
                       double* vbar, uint8_t* reason, int64_t* undo_iterations) {
  return guarded(c, [&]() -> pamo_status {
    if (!V || !F || !cand || !ncand || !vbar || !reason) fail(PAMO_ERR_ARG, "null pointer");
    check_sizes(nv, nf);
    if (target_faces < 0) fail(PAMO_ERR_ARG, "negative target");
    reserve(c, nv, nf, Parts{});
    MeshView A = mesh_bufs(c->ws, "mA", nv, nf);
    load_mesh(c, A, V, F, flags);
    RoundBufs b = round_bufs(c->ws, nv, nf);
    int nc = read_count(c, ncand);
    // chosen edges have disjoint rings of at least two faces each
    if (nc < 0 || nc > nf / 2 + 1) fail(PAMO_ERR_ARG, "bad candidate count (more than nf / 2 + 1)");
    if (undo_iterations) *undo_iterations = 0;
    if (nc == 0) return PAMO_OK;
    hipStream_t s = c->stream;
    fill_i32(s, c->dcnt, C_COUNT, 0);
    launch_quadrics(s, A, b.Q, c->dcnt + C_ERR);
    launch_cost_keys(c->ws, s, A, b.Q, c->opt.w_e, c->opt.w_s, nullptr, nullptr, b.key, c->dcnt + C_ERR,
                     c->opt.cost_target, false, c->opt.key_mode != 0);
    if (c->opt.key_mode) launch_rank_keys(c->ws, s, A, b.key);  // the cap orders by key
    int64_t teff = target_faces - target_faces % 2;
    if (A.nf <= teff) fail(PAMO_ERR_ARG, "the mesh is already at or below the target");
    RoundResult R;
    R.ncand = nc;
    local_checks(c, A, b, cand, ncand, nc, reason, vbar);
    const int* h = readback(c);
    check_err_bits(h[C_ERR]);
    R.npass = h[C_HIST + 0];
    prof_bytes(c, PH_LOCAL, 780.0 * nc);
    cap_single(c, b, ncand, reason, teff, A.nf, R);
    check_and_undo(c, A, b, cand, ncand, nc, reason, vbar, R, nullptr);
    fill_u8(s, b.valive, A.nv, 1);
    if (R.chosen > 0) launch_commit(s, A, cand, ncand, nc, reason, b.undone, b.valive);
    check_err_bits(readback(c)[C_ERR]);
    if (undo_iterations) *undo_iterations = R.iters;
    return PAMO_OK;
  });
}

pamo_status pamo_collapse(pamo_ctx* c, double* V, int64_t* nv, int32_t* F, int64_t* nf, const int32_t* cand,
                          const int32_t* ncand, const double* vbar, const uint8_t* reason, uint8_t* flags_io) {
  return guarded(c, [&]() -> pamo_status {
    if (!V || !nv || !F || !nf || !cand || !ncand || !vbar || !reason) fail(PAMO_ERR_ARG, "null pointer");
    check_sizes(*nv, *nf);
    reserve(c, *nv, *nf, Parts{});
    hipStream_t s = c->stream;
    MeshView A = mesh_bufs(c->ws, "mA", *nv, *nf);
    MeshView B = mesh_bufs(c->ws, "mB", *nv, *nf);
    load_mesh(c, A, V, F, flags_io);
    RoundBufs b = round_bufs(c->ws, *nv, *nf);
    int nc = read_count(c, ncand);
    if (nc < 0 || nc > 3 * *nf) fail(PAMO_ERR_ARG, "bad candidate count");
    int* cnt = c->dcnt;
    fill_i32(s, cnt, C_COUNT, 0);
    int commits = 0;
    if (nc > 0) {
      PAMO_HIP(hipMemcpyAsync(b.reason, reason, nc, hipMemcpyDeviceToDevice, s));
      fill_u8(s, b.falive, A.nf, 1);
      fill_u8(s, b.valive, A.nv, 1);
      fill_i32(s, b.owner, A.nf, -1);
      fill_i32(s, b.undone, nc, 0);
      launch_face_boxes(s, A, b.box);
      launch_apply(s, A, cand, ncand, nc, b.reason, vbar, b.oldpos, b.owner, b.falive, b.box);
      launch_commit(s, A, cand, ncand, nc, b.reason, b.undone, b.valive);
      launch_reason_hist(s, ncand, nc, b.reason, cnt + C_HIST2);
      commits = readback(c)[C_HIST2];
      if (commits > 0) fill_u8(s, A.flags, 3 * (int64_t)A.nf, 0);
      launch_flags(s, A, cand, ncand, nc, b.reason);
    }
    if (commits > 0) {
      launch_compact(c->ws, s, A, B, b.falive, b.valive, cnt + C_NF, cnt + C_NV, cnt + C_ERR);
      const int* h = readback(c);
      check_err_bits(h[C_ERR]);
      B.nf = h[C_NF];
      B.nv = h[C_NV];
      PAMO_HIP(hipMemcpyAsync(V, B.V, 3 * (size_t)B.nv * sizeof(double), hipMemcpyDeviceToDevice, s));
      PAMO_HIP(hipMemcpyAsync(F, B.F, 3 * (size_t)B.nf * sizeof(int), hipMemcpyDeviceToDevice, s));
      if (flags_io) PAMO_HIP(hipMemcpyAsync(flags_io, B.flags, 3 * (size_t)B.nf, hipMemcpyDeviceToDevice, s));
      *nv = B.nv;
      *nf = B.nf;
    } else if (flags_io) {
      PAMO_HIP(hipMemcpyAsync(flags_io, A.flags, 3 * (size_t)A.nf, hipMemcpyDeviceToDevice, s));
    }
    PAMO_HIP(hipStreamSynchronize(s));
    return PAMO_OK;
  });
}

pamo_status pamo_simplify(pamo_ctx* c, const double* V, int64_t nv, const int32_t* F, int64_t nf,
                          int64_t target_faces, double* V_out, int64_t* nv_out, int32_t* F_out, int64_t* nf_out,
                          pamo_stats* stats) {
  return guarded(c, [&]() -> pamo_status {
    if (!V || !F || !V_out || !F_out || !nv_out || !nf_out) fail(PAMO_ERR_ARG, "null pointer");
    LearnRun L;
    L.learned = c->opt.learned != 0;
    L.track = L.learned;
    return simplify_run(c, V, nv, F, nf, target_faces, V_out, nv_out, F_out, nf_out, stats, &L);
  });
}

pamo_status pamo_simplify_noalloc(pamo_ctx* c, const double* V, int64_t nv, const int32_t* F, int64_t nf,
                                  int64_t target_faces, double* V_out, int64_t* nv_out, int32_t* F_out,
                                  int64_t* nf_out, pamo_stats* stats) {
  if (!c) return PAMO_ERR_ARG;
  // For this call the context's workspace is the device's static scratch: the
  // context's own buffers are set aside (a swap of host bookkeeping) and come
  // back afterwards; phase timing (HIP events) is off.
  Workspace arena;
  arena.arena = static_cast<char*>(c->scratch);
  arena.arena_bytes = c->scratch ? (size_t)PAMO_NOALLOC_SCRATCH_BYTES : 0;
  std::swap(c->ws, arena);
  int* const own_cnt = c->dcnt;
  const uint32_t mask = c->prof.mask;
  c->prof.mask = 0;
  const pamo_status rc = guarded(c, [&]() -> pamo_status {
    if (!c->scratch) fail(PAMO_ERR_HIP, "no static scratch on this device");
    if (!V || !F || !V_out || !F_out || !nv_out || !nf_out) fail(PAMO_ERR_ARG, "null pointer");
    check_sizes(nv, nf);
    LearnRun L;
    L.learned = c->opt.learned != 0;
    L.track = L.learned;
    Workspace count;  // what this call reserves, summed on the host
    count.counting = true;
    count.get<int>("ctx.cnt", C_COUNT);
    Parts parts;
    parts.learned = L.track;
    reserve_mesh(count, nv, nf, c->opt, parts);
    if (count.total > (size_t)PAMO_NOALLOC_SCRATCH_BYTES)
      fail(PAMO_ERR_CAPACITY, "pamo_simplify_noalloc: the mesh needs " + std::to_string(count.total) +
                                  " bytes of scratch, more than the " + std::to_string(PAMO_NOALLOC_SCRATCH_BYTES) +
                                  " of the static scratch");
    return simplify_run(c, V, nv, F, nf, target_faces, V_out, nv_out, F_out, nf_out, stats, &L);
  });
  std::swap(c->ws, arena);
  c->dcnt = own_cnt;
  c->prof.mask = mask;
  return rc;
}

pamo_status pamo_collect(pamo_ctx* c, const double* V, int64_t nv, const int32_t* F, int64_t nf,
                         int64_t target_faces, float* X, uint8_t* y, int64_t cap, int64_t* rows, pamo_stats* stats) {
  return guarded(c, [&]() -> pamo_status {
    if (!V || !F || !rows || cap < 0 || (cap > 0 && (!X || !y))) fail(PAMO_ERR_ARG, "bad arguments");
    if (c->opt.key_mode || c->opt.prefilter)
      fail(PAMO_ERR_ARG, "training rows come from the plain selection with float32 keys (key_mode 0, prefilter 0)");
    LearnRun L;
    L.track = true;
    L.X = cap > 0 ? X : nullptr;
    L.y = y;
    L.cap = cap;
    double* Vo = c->ws.get<double>("col.V", 3 * nv);
    int* Fo = c->ws.get<int>("col.F", 3 * nf);
    int64_t nvo = 0, nfo = 0;
    pamo_status st = simplify_run(c, V, nv, F, nf, target_faces, Vo, &nvo, Fo, &nfo, stats, &L);
    *rows = L.n;
    return st;
  });
}

pamo_status pamo_simplify_batch(pamo_ctx* c, int32_t nmesh, const double* V, const int64_t* v_off, const int32_t* F,
                                const int64_t* f_off, const int64_t* targets, double* V_out, int64_t* v_out_off,
                                int32_t* F_out, int64_t* f_out_off, pamo_stats* stats) {
  return guarded(c, [&]() -> pamo_status {
    if (!V || !v_off || !F || !f_off || !targets || !V_out || !v_out_off || !F_out || !f_out_off)
      fail(PAMO_ERR_ARG, "null pointer");
    if (nmesh < 1 || nmesh > PAMO_MAX_MESHES) fail(PAMO_ERR_ARG, "nmesh must be in [1, 4096]");
    if (v_off[0] != 0 || f_off[0] != 0) fail(PAMO_ERR_ARG, "offsets must start at 0");
    for (int m = 0; m < nmesh; m++) {
      if (v_off[m + 1] - v_off[m] < 4 || f_off[m + 1] - f_off[m] < 4)
        fail(PAMO_ERR_ARG, "mesh " + std::to_string(m) + ": a closed mesh needs at least 4 vertices and 4 faces");
      if (targets[m] < 0) fail(PAMO_ERR_ARG, "mesh " + std::to_string(m) + ": negative target");
    }
    const int64_t nv = v_off[nmesh], nf = f_off[nmesh];
    check_sizes(nv, nf);
    Parts parts;
    parts.nmesh = std::max(nmesh, 2);
    parts.learned = c->opt.learned != 0;
    reserve(c, nv, nf, parts);
    hipStream_t s = c->stream;
    MeshView cur = mesh_bufs(c->ws, "mA", nv, nf);
    MeshView alt = mesh_bufs(c->ws, "mB", nv, nf);
    cur.fmesh = c->ws.get<int>("mA.fmesh", nf);
    cur.vmesh = c->ws.get<int>("mA.vmesh", nv);
    alt.fmesh = c->ws.get<int>("mB.fmesh", nf);
    alt.vmesh = c->ws.get<int>("mB.vmesh", nv);
    Batch B = batch_bufs(c, nmesh);
    for (int m = 0; m <= nmesh; m++) {
      c->hbt[B.f_off() + m] = (int)f_off[m];
      c->hbt[B.v_off() + m] = (int)v_off[m];
    }
    PAMO_HIP(hipMemcpyAsync(B.d(B.f_off()), c->hbt + B.f_off(), (size_t)(2 * nmesh + 2) * sizeof(int),
                            hipMemcpyHostToDevice, s));
    PAMO_HIP(hipMemcpyAsync(cur.V, V, 3 * (size_t)nv * sizeof(double), hipMemcpyDeviceToDevice, s));
    PAMO_HIP(hipMemcpyAsync(cur.F, F, 3 * (size_t)nf * sizeof(int), hipMemcpyDeviceToDevice, s));
    fill_i32(s, c->dcnt, C_COUNT, 0);
    launch_batch_ids(s, B.d(B.f_off()), B.d(B.v_off()), nmesh, (int)nf, (int)nv, cur.F, cur.fmesh, cur.vmesh,
                     c->dcnt + C_ERR);
    fill_u8(s, cur.flags, 3 * nf, 0);
    launch_adjacency(c->ws, s, cur, c->dcnt + C_ERR);
    check_err_bits(readback(c)[C_ERR]);
    launch_check_vertices(c->ws, s, cur, c->dcnt + C_ERR);
    check_err_bits(readback(c)[C_ERR]);
    if (c->opt.validate_input) {
      int2* dummy = c->ws.get<int2>("w.pairs", 1);
      if (whole_mesh_pairs(c, cur, dummy, 0, nmesh) > 0) fail(PAMO_ERR_SELF_INTERSECTING, "an input mesh intersects itself");
    }
    RoundBufs b = round_bufs(c->ws, nv, nf);
    const bool learned = c->opt.learned != 0;
    if (learned && !c->mlp) fail(PAMO_ERR_ARG, "the learned proposal needs a network (pamo_set_mlp)");
    if (learned && c->opt.key_mode)
      fail(PAMO_ERR_ARG, "the learned proposal's features read the float32 cost from the key (key_mode 0)");
    if (learned) {
      cur.ovl = c->ws.get<int>("mA.ovl", nf);
      alt.ovl = c->ws.get<int>("mB.ovl", nf);
      b.ovl_new = c->ws.get<int>("r.ovl_new", nf);
      b.X = c->ws.get<float>("r.X", (nf / 2 + 1) * (int64_t)LEARN_NFEAT);
      b.dlist = c->ws.get<int>("r.dlist", nf / 2 + 1);
      int2* dummy = c->ws.get<int2>("w.pairs", 1);
      whole_mesh_pairs(c, cur, dummy, 0, nmesh, cur.ovl);
    }
    std::vector<MeshRun> mr(nmesh);
    for (int m = 0; m < nmesh; m++) mr[m].teff = targets[m] - targets[m] % 2;
    int64_t deferred = 0;
    OrderState os;
    os.resort = c->opt.resort_every > 0 ? c->opt.resort_every : PAMO_DEFAULT_RESORT;
    bool any_unreached = false;
    for (;;) {
      int nactive = 0;
      for (int m = 0; m < nmesh; m++) {
        MeshRun& r = mr[m];
        r.active = false;
        if (r.st.status != PAMO_OK || r.settled) continue;
        int64_t nfm = c->hbt[B.f_off() + m + 1] - c->hbt[B.f_off() + m];
        if (nfm <= r.teff) continue;
        if (r.streak >= c->opt.tolerance) {
          r.st.status = PAMO_TARGET_UNREACHED;
          any_unreached = true;
          continue;
        }
        if (c->opt.max_rounds >= 0 && r.st.rounds >= c->opt.max_rounds) continue;
        r.active = true;
        nactive++;
      }
      if (nactive == 0) break;
      RoundResult R = run_round_batch(c, cur, alt, b, B, mr, os, learned, learned);
      deferred += R.deferred;
      // per-mesh outcome of the round (tallies in the host mirror)
      auto absorb = [&](int m) {
        MeshRun& r = mr[m];
        int ncm = c->hbt[B.ncand_m() + m];
        int cm = c->hbt[B.commits_m() + m];
        const int* hm = c->hbt + B.hist_m() + 8 * m;
        r.st.rounds++;
        r.st.candidates += ncm;
        r.st.commits += cm;
        r.st.rej_link += hm[1];
        r.st.rej_flip += hm[2];
        r.st.rej_isect += hm[3];
        r.st.capped += hm[4];
        r.st.undo_hist[std::min(c->hbt[B.undo_m() + m], 4)]++;
        r.streak = cm == 0 ? r.streak + 1 : 0;
        r.rejected = hm[1] + hm[2] + hm[3] > 0;
        if (c->opt.cost_target > 0 && ncm == 0) r.settled = true;
      };
      std::vector<int> retry;
      for (int m = 0; m < nmesh; m++) {
        if (!mr[m].active) continue;
        const int dm = c->hbt[B.demote_m() + m];
        mr[m].st.demoted += dm;
        if (learned && dm > 0 && c->hbt[B.commits_m() + m] == 0) {
          retry.push_back(m);  // set candidates aside and committed nothing: run it again plain
          continue;
        }
        absorb(m);
      }
      if (!retry.empty()) {
        for (int m = 0; m < nmesh; m++) mr[m].active = false;
        for (int m : retry) mr[m].active = true;
        RoundResult R2 = run_round_batch(c, cur, alt, b, B, mr, os, false, learned);
        deferred += R2.deferred;
        for (int m : retry) {
          mr[m].st.fallbacks++;
          absorb(m);
        }
      }
    }
    launch_batch_output(s, cur, B.d(B.f_off()), B.d(B.v_off()), B.d(B.f_off()), B.d(B.v_off()), nmesh, V_out, F_out);
    PAMO_HIP(hipStreamSynchronize(s));
    for (int m = 0; m <= nmesh; m++) {
      f_out_off[m] = c->hbt[B.f_off() + m];
      v_out_off[m] = c->hbt[B.v_off() + m];
    }
    if (stats) {
      for (int m = 0; m < nmesh; m++) {
        pamo_stats& o = stats[m];
        o = mr[m].st;
        o.faces_out = f_out_off[m + 1] - f_out_off[m];
        o.verts_out = v_out_off[m + 1] - v_out_off[m];
        o.deferred_pairs = deferred;
      }
    }
    return any_unreached ? PAMO_TARGET_UNREACHED : PAMO_OK;
  });
}

// ------------------------------------------------------------ learned proposal
static bool on_grid(float w, int e, double kmax) {
  double k = ldexp((double)w, e);
  return k == rint(k) && fabs(k) <= kmax;
}

pamo_status pamo_set_mlp(pamo_ctx* c, const pamo_mlp* m) {
  return guarded(c, [&]() -> pamo_status {
    if (!m) {
      if (c->mlp) PAMO_HIP(hipFree(c->mlp));
      c->mlp = nullptr;
      return PAMO_OK;
    }
    const int e[3] = {m->e1, m->e2, m->e3};
    for (int l = 0; l < 3; l++)
      if (e[l] < 0 || e[l] > 15) fail(PAMO_ERR_ARG, "weight grid exponent outside [0, 15]");
    if (m->a1 < -30 || m->a1 > 30 || m->a2 < -30 || m->a2 > 30) fail(PAMO_ERR_ARG, "activation shift outside [-30, 30]");
    const double BMAX = 4194304.0;  // 2^22
    for (int j = 0; j < 64; j++) {
      for (int k = 0; k < 32; k++)
        if (!on_grid(m->w1[j][k], e[0], 127)) fail(PAMO_ERR_ARG, "w1 off its grid");
      for (int k = 0; k < 64; k++)
        if (!on_grid(m->w2[j][k], e[1], 127)) fail(PAMO_ERR_ARG, "w2 off its grid");
      if (!on_grid(m->w3[j], e[2], 127)) fail(PAMO_ERR_ARG, "w3 off its grid");
      if (!on_grid(m->b1[j], e[0], BMAX) || !on_grid(m->b2[j], e[1], BMAX)) fail(PAMO_ERR_ARG, "bias off its grid");
    }
    if (!on_grid(m->b3, e[2], BMAX)) fail(PAMO_ERR_ARG, "bias off its grid");
    if (!(m->threshold == m->threshold)) fail(PAMO_ERR_ARG, "threshold is NaN");
    MlpDev h;
    memset(&h, 0, sizeof(h));
    // grid values have at most 7 significant bits: bfloat16 holds them
    // exactly, as the upper half of their float32 bits
    auto bf = [](float x) {
      uint32_t u;
      memcpy(&u, &x, 4);
      return (uint16_t)(u >> 16);
    };
    uint16_t* w1 = reinterpret_cast<uint16_t*>(h.w1);
    uint16_t* w2 = reinterpret_cast<uint16_t*>(h.w2);
    for (int j = 0; j < 64; j++) {
      for (int k = 0; k < 32; k++) w1[j * 32 + k] = bf(m->w1[j][k]);
      for (int k = 0; k < 64; k++) w2[j * 64 + k] = bf(m->w2[j][k]);
      h.w3[j] = m->w3[j];
      h.b1[j] = m->b1[j];
      h.b2[j] = m->b2[j];
    }
    h.b3 = m->b3;
    h.a1 = m->a1;
    h.a2 = m->a2;
    h.threshold = m->threshold;
    if (!c->mlp) PAMO_HIP(hipMalloc((void**)&c->mlp, sizeof(MlpDev)));
    PAMO_HIP(hipMemcpyAsync(c->mlp, &h, sizeof(MlpDev), hipMemcpyHostToDevice, c->stream));
    PAMO_HIP(hipStreamSynchronize(c->stream));
    return PAMO_OK;
  });
}

pamo_status pamo_features(pamo_ctx* c, const double* V, int64_t nv, const int32_t* F, int64_t nf,
                          const int32_t* edges, int64_t ne, float* X, int32_t* ovl) {
  return guarded(c, [&]() -> pamo_status {
    if (!V || !F || ne < 0 || (ne > 0 && (!edges || !X))) fail(PAMO_ERR_ARG, "bad arguments");
    check_sizes(nv, nf);
    if (ne > 3 * nf) fail(PAMO_ERR_ARG, "more edges than half-edges");
    if (c->opt.key_mode) fail(PAMO_ERR_ARG, "the features read the float32 cost from the key (key_mode 0)");
    Parts parts;
    parts.learned = true;
    reserve(c, nv, nf, parts);
    hipStream_t s = c->stream;
    MeshView A = mesh_bufs(c->ws, "mA", nv, nf);
    load_mesh(c, A, V, F, nullptr);
    A.ovl = c->ws.get<int>("mA.ovl", nf);
    int2* dummy = c->ws.get<int2>("w.pairs", 1);
    whole_mesh_pairs(c, A, dummy, 0, 1, A.ovl);
    RoundBufs b = round_bufs(c->ws, nv, nf);
    fill_i32(s, c->dcnt, C_COUNT, 0);
    if (ne > 0) {
      hipLaunchKernelGGL(k_check_index, dim3(nblk(ne)), dim3(256), 0, s, edges, ne, (int)(3 * nf), c->dcnt + C_ERR);
      check_err_bits(readback(c)[C_ERR]);
      A.vstar = b.vstar;  // the stored stars, as in a round
      A.vdeg = b.vdeg;
      A.vbox = b.vbox;
      launch_quadrics(s, A, b.Q, c->dcnt + C_ERR);
      launch_cost_keys(c->ws, s, A, b.Q, c->opt.w_e, c->opt.w_s, nullptr, nullptr, b.key, c->dcnt + C_ERR,
                     c->opt.cost_target);
      fill_i32(s, c->dcnt + C_NCAND, 1, (int)ne);
      launch_features(s, A, b.key, edges, c->dcnt + C_NCAND, (int)ne, A.ovl, X, c->dcnt + C_ERR);
    }
    if (ovl) PAMO_HIP(hipMemcpyAsync(ovl, A.ovl, (size_t)nf * sizeof(int), hipMemcpyDeviceToDevice, s));
    check_err_bits(readback(c)[C_ERR]);
    return PAMO_OK;
  });
}

pamo_status pamo_mlp_logits(pamo_ctx* c, const float* X, int64_t n, float* logits) {
  return guarded(c, [&]() -> pamo_status {
    if (!c->mlp) fail(PAMO_ERR_ARG, "no network set");
    if (n < 0 || n > INT32_MAX || (n > 0 && (!X || !logits))) fail(PAMO_ERR_ARG, "bad arguments");
    if (n == 0) return PAMO_OK;
    int* nd = c->ws.get<int>("mlp.n", 1);
    fill_i32(c->stream, nd, 1, (int)n);
    launch_mlp(c->stream, X, nd, (int)n, c->mlp, logits, nullptr, nullptr, nullptr, nullptr);
    return PAMO_OK;
  });
}

static MlpMeta meta_of(const int32_t* m) {
  if (!m) fail(PAMO_ERR_ARG, "null meta");
  for (int l = 0; l < 3; l++)
    if (m[l] < 0 || m[l] > 15) fail(PAMO_ERR_ARG, "weight grid exponent outside [0, 15]");
  if (m[3] < -30 || m[3] > 30 || m[4] < -30 || m[4] > 30) fail(PAMO_ERR_ARG, "activation shift outside [-30, 30]");
  return MlpMeta{m[0], m[1], m[2], m[3], m[4]};
}

pamo_status pamo_mlp_grad(pamo_ctx* c, const float* params, const int32_t* meta, const float* X, const uint8_t* y,
                          int64_t n, float* grad, float* loss) {
  return guarded(c, [&]() -> pamo_status {
    MlpMeta md = meta_of(meta);
    if (!params || !X || !y || !grad || n < 1 || n > (1 << 18)) fail(PAMO_ERR_ARG, "bad arguments (1 <= n <= 2^18)");
    hipStream_t s = c->stream;
    int nb = (int)n, blocks = train_blocks(nb);
    float* part = c->ws.get<float>("tr.part", (int64_t)blocks * LEARN_NPARAM);
    float* ploss = c->ws.get<float>("tr.ploss", blocks);
    float* dloss = c->ws.get<float>("tr.loss", 1);
    launch_train_grad(s, params, md, X, y, nullptr, 0, nb, n, part, ploss);
    launch_train_reduce(s, part, ploss, nb, md, const_cast<float*>(params), grad, nullptr, nullptr, 0.0f, 0, dloss);
    float l = 0;
    PAMO_HIP(hipMemcpyAsync(&l, dloss, sizeof(float), hipMemcpyDeviceToHost, s));
    PAMO_HIP(hipStreamSynchronize(s));
    if (loss) *loss = l;
    return PAMO_OK;
  });
}

pamo_status pamo_mlp_train(pamo_ctx* c, float* params, float* m, float* v, const int32_t* meta, const float* X,
                           const uint8_t* y, int64_t n, const int32_t* order, int64_t steps, int64_t batch, float lr,
                           int64_t t0, float* loss) {
  return guarded(c, [&]() -> pamo_status {
    MlpMeta md = meta_of(meta);
    if (!params || !m || !v || !X || !y || !order || n < 1 || steps < 0 || batch < 1 || batch > (1 << 16) || t0 < 0)
      fail(PAMO_ERR_ARG, "bad arguments (1 <= batch <= 2^16)");
    hipStream_t s = c->stream;
    int nb = (int)batch, blocks = train_blocks(nb);
    float* part = c->ws.get<float>("tr.part", (int64_t)blocks * LEARN_NPARAM);
    float* ploss = c->ws.get<float>("tr.ploss", blocks);
    float* dloss = c->ws.get<float>("tr.loss", 1);
    for (int64_t st = 0; st < steps; st++) {
      launch_train_grad(s, params, md, X, y, order, st * batch, nb, n, part, ploss);
      launch_train_reduce(s, part, ploss, nb, md, params, nullptr, m, v, lr, t0 + st + 1, loss ? loss + st : dloss);
    }
    return PAMO_OK;
  });
}

pamo_status pamo_hausdorff(pamo_ctx* c, const double* P, int64_t np, const double* V, int64_t nv, const int32_t* F,
                           int64_t nf, double* dist, double* dmax) {
  return guarded(c, [&]() -> pamo_status {
    if (!P || !V || !F || !dmax || np < 0 || np > INT32_MAX || nv < 1 || nf < 1 || nf > INT32_MAX / 3)
      fail(PAMO_ERR_ARG, "bad arguments");
    hipStream_t s = c->stream;
    fill_i32(s, c->dcnt, C_COUNT, 0);
    hipLaunchKernelGGL(k_check_index, dim3(nblk(3 * nf)), dim3(256), 0, s, F, 3 * nf, (int)nv, c->dcnt + C_ERR);
    check_err_bits(readback(c)[C_ERR]);
    uint64_t* bits = c->ws.get<uint64_t>("hd.max", 1);
    fill_i32(s, reinterpret_cast<int32_t*>(bits), 2, 0);
    if (np > 0) launch_point_surface(s, P, (int)np, V, F, (int)nf, dist, bits);
    uint64_t hb = 0;
    PAMO_HIP(hipMemcpyAsync(&hb, bits, sizeof(hb), hipMemcpyDeviceToHost, s));
    PAMO_HIP(hipStreamSynchronize(s));
    memcpy(dmax, &hb, sizeof(double));
    return PAMO_OK;
  });
}

constexpr int64_t kUdfScanMax = (int64_t)1 << 26;

pamo_status pamo_udf(pamo_ctx* c, const double* V, int64_t nv, const int32_t* F, int64_t nf, int32_t res, double band,
                     double* udf) {
  return guarded(c, [&]() -> pamo_status {
    if (!udf || (nf > 0 && (!V || !F))) fail(PAMO_ERR_ARG, "null pointer");
    if (nv < 0 || nf < 0 || nf > (int64_t)(INT32_MAX / 3) - 1 || (nf > 0 && nv < 1)) fail(PAMO_ERR_ARG, "bad sizes");
    if (res < 1 || res > 2048) fail(PAMO_ERR_ARG, "grid resolution outside [1, 2048]");
    if (!(band > 0.0) || !(band < INFINITY)) fail(PAMO_ERR_ARG, "band width must be positive and finite");
    // the library's scans take at most 2^26 items: the per-triangle pair counts
    // and the per-pair run flags are scanned whole
    if (nf > kUdfScanMax) fail(PAMO_ERR_CAPACITY, "more than 2^26 triangles for the distance field");
    hipStream_t s = c->stream;
    fill_i32(s, c->dcnt, C_COUNT, 0);
    if (nf > 0) {
      hipLaunchKernelGGL(k_check_index, dim3(nblk(3 * nf)), dim3(256), 0, s, F, 3 * nf, (int)nv, c->dcnt + C_ERR);
      check_err_bits(readback(c)[C_ERR]);
    }
    udf_run(c->ws, s, V, F, (int)nf, res, band, udf, c->dcnt + C_ERR, [&](const unsigned long long* total) {
      unsigned long long t = 0;
      PAMO_HIP(hipMemcpyAsync(&t, total, sizeof(t), hipMemcpyDeviceToHost, s));
      check_err_bits(readback(c)[C_ERR]);  // synchronises
      if (t > (unsigned long long)kUdfScanMax) fail(PAMO_ERR_CAPACITY, "more than 2^26 tile-triangle pairs");
      return (int64_t)t;
    });
    PAMO_HIP(hipStreamSynchronize(s));
    return PAMO_OK;
  });
}

pamo_status pamo_dualmc(pamo_ctx* c, const double* S, int32_t res, double iso, double beta, double* V_out,
                        int64_t vcap, int32_t* F_out, int64_t fcap, int64_t* nv_out, int64_t* nf_out) {
  return guarded(c, [&]() -> pamo_status {
    if (!S || !nv_out || !nf_out || (vcap > 0 && !V_out) || (fcap > 0 && !F_out)) fail(PAMO_ERR_ARG, "null pointer");
    if (res < 2 || res > 512) fail(PAMO_ERR_ARG, "grid resolution outside [2, 512]");
    if (vcap < 0 || fcap < 0 || !(iso == iso)) fail(PAMO_ERR_ARG, "bad sizes or iso value");
    if (!(beta >= 0.0) || !(beta < INFINITY)) fail(PAMO_ERR_ARG, "beta must be finite and >= 0");
    if (!dualmc_run(c->ws, c->stream, S, res, iso, beta, V_out, vcap, F_out, fcap, nv_out, nf_out))
      fail(PAMO_ERR_CAPACITY, "output capacity too small for the extracted mesh");
    PAMO_HIP(hipStreamSynchronize(c->stream));
    return PAMO_OK;
  });
}

void pamo_project_defaults(pamo_project_options* o) {
  if (!o) return;
  o->k_dis = 1e3;
  o->k_elas = 1e-1;
  o->k_bend = 1e-2;
  o->k_bar = 1e2;
  o->dhat = 1e-3;
  o->cg_tol = 1e-4;
  o->accd_s = 0.1;
  o->iterations = 50;
  o->refresh = 10;
  o->cg_max = 1000;
  o->ls_max = 40;
}

namespace {
pamo_project_options project_options(const pamo_project_options* opt) {
  pamo_project_options o;
  pamo_project_defaults(&o);
  if (opt) o = *opt;
  auto fin = [](double x) { return x == x && x < INFINITY && x > -INFINITY; };
  if (!fin(o.k_dis) || !fin(o.k_elas) || !fin(o.k_bend) || !fin(o.k_bar) || o.k_dis < 0 || o.k_elas < 0 ||
      o.k_bend < 0 || o.k_bar < 0)
    fail(PAMO_ERR_ARG, "energy weights must be finite and >= 0");
  if (!fin(o.dhat) || !(o.dhat > 0)) fail(PAMO_ERR_ARG, "dhat must be positive");
  if (!fin(o.cg_tol) || !(o.cg_tol > 0) || o.cg_max < 1) fail(PAMO_ERR_ARG, "bad CG options");
  if (!(o.accd_s > 0 && o.accd_s < 1)) fail(PAMO_ERR_ARG, "accd_s must lie in (0, 1)");
  if (o.iterations < 0 || o.refresh < 1 || o.ls_max < 1) fail(PAMO_ERR_ARG, "bad iteration options");
  return o;
}

void check_faces(pamo_ctx* c, const int32_t* F, int64_t nf, int64_t nv) {
  if (nf <= 0) return;
  fill_i32(c->stream, c->dcnt, C_COUNT, 0);
  hipLaunchKernelGGL(k_check_index, dim3(nblk(3 * nf)), dim3(256), 0, c->stream, F, 3 * nf, (int)nv, c->dcnt + C_ERR);
  check_err_bits(readback(c)[C_ERR]);
}

void check_mesh_sizes(int64_t nv, int64_t nf, int64_t min_nf) {
  if (nv < 1 || nf < min_nf || nf > (int64_t)(INT32_MAX / 9) || nv > (int64_t)(INT32_MAX / 9))
    fail(PAMO_ERR_ARG, "bad sizes");
}
}  // namespace

pamo_status pamo_sample_surface(pamo_ctx* c, const double* V, int64_t nv, const int32_t* F, int64_t nf,
                                const double* U, int64_t m, double* Y, double* area) {
  return guarded(c, [&]() -> pamo_status {
    if (!V || !F || (m > 0 && (!U || !Y))) fail(PAMO_ERR_ARG, "null pointer");
    check_mesh_sizes(nv, nf, 1);
    if (m < 0 || m > (int64_t)(INT32_MAX / 3)) fail(PAMO_ERR_ARG, "bad sample count");
    check_faces(c, F, nf, nv);
    const double a = project_sample(c->ws, c->stream, V, (int)nv, F, (int)nf, U, m, Y);
    if (area) *area = a;
    return PAMO_OK;
  });
}

pamo_status pamo_project_targets(pamo_ctx* c, const double* X, int64_t nv, const int32_t* F, int64_t nf,
                                 const double* Vin, int64_t nv_in, const int32_t* Fin, int64_t nf_in, const double* Y,
                                 int64_t m, double* targets, int32_t* tri) {
  return guarded(c, [&]() -> pamo_status {
    if (!X || !F || !Vin || !Fin || !targets || (m > 0 && (!Y || !tri))) fail(PAMO_ERR_ARG, "null pointer");
    check_mesh_sizes(nv, nf, 1);
    check_mesh_sizes(nv_in, nf_in, 1);
    if (m < 0 || m > (int64_t)(INT32_MAX / 3)) fail(PAMO_ERR_ARG, "bad sample count");
    check_faces(c, F, nf, nv);
    check_faces(c, Fin, nf_in, nv_in);
    project_targets(c->ws, c->stream, X, (int)nv, F, (int)nf, Vin, (int)nv_in, Fin, (int)nf_in, Y, (int)m, targets,
                    tri);
    return PAMO_OK;
  });
}

pamo_status pamo_project_eval(pamo_ctx* c, const double* X0, const double* X, int64_t nv, const int32_t* F,
                              int64_t nf, const double* targets, const double* Y, const int32_t* tri, int64_t m,
                              double area_in, const pamo_project_options* opt, double* parts, int64_t* contacts,
                              double* grad, const double* v, double* Hv, double* dir, int32_t* cg_iters, double* step) {
  return guarded(c, [&]() -> pamo_status {
    if (!X0 || !X || !F || !targets || !parts || (m > 0 && (!Y || !tri)) || (Hv && !v) || (step && !dir))
      fail(PAMO_ERR_ARG, "null pointer");
    check_mesh_sizes(nv, nf, 4);
    if (m < 0 || m > (int64_t)(INT32_MAX / 3)) fail(PAMO_ERR_ARG, "bad sample count");
    if (!(area_in >= 0) || !(area_in < INFINITY)) fail(PAMO_ERR_ARG, "bad input area");
    const pamo_project_options o = project_options(opt);
    check_faces(c, F, nf, nv);
    if (m > 0) {  // the samples' triangles must exist
      fill_i32(c->stream, c->dcnt, C_COUNT, 0);
      hipLaunchKernelGGL(k_check_index, dim3(nblk(m)), dim3(256), 0, c->stream, tri, m, (int)nf, c->dcnt + C_ERR);
      check_err_bits(readback(c)[C_ERR]);
    }
    ProjectEvalOut out;
    out.grad = grad;
    out.v = v;
    out.Hv = Hv;
    out.dir = dir;
    out.want_step = step != nullptr;
    try {
      project_eval(c->ws, c->stream, X0, X, (int)nv, F, (int)nf, targets, Y, tri, (int)m, area_in, o, out);
    } catch (const ProjectMeshError& e) {
      fail(PAMO_ERR_NONMANIFOLD, e.what());
    }
    for (int k = 0; k < 6; k++) parts[k] = out.parts[k];
    if (contacts) {
      contacts[0] = out.npt;
      contacts[1] = out.nee;
    }
    if (cg_iters) *cg_iters = out.cg_iters;
    if (step) *step = out.step;
    return PAMO_OK;
  });
}

pamo_status pamo_safe_project(pamo_ctx* c, const double* Vs, int64_t nv, const int32_t* Fs, int64_t nf,
                              const double* Vin, int64_t nv_in, const int32_t* Fin, int64_t nf_in, const double* Y,
                              int64_t m, const pamo_project_options* opt, double* V_out, double* log,
                              pamo_project_stats* stats) {
  return guarded(c, [&]() -> pamo_status {
    if (!Vs || !Fs || !Vin || !Fin || !V_out || (m > 0 && !Y)) fail(PAMO_ERR_ARG, "null pointer");
    check_mesh_sizes(nv, nf, 4);
    check_mesh_sizes(nv_in, nf_in, 1);
    if (m < 0 || m > (int64_t)(INT32_MAX / 3)) fail(PAMO_ERR_ARG, "bad sample count");
    const pamo_project_options o = project_options(opt);
    check_faces(c, Fs, nf, nv);
    check_faces(c, Fin, nf_in, nv_in);
    try {
      project_run(c->ws, c->stream, Vs, (int)nv, Fs, (int)nf, Vin, (int)nv_in, Fin, (int)nf_in, Y, (int)m, o, V_out,
                  log, stats);
    } catch (const ProjectMeshError& e) {
      fail(PAMO_ERR_NONMANIFOLD, e.what());
    }
    return PAMO_OK;
  });
}

pamo_status pamo_self_intersections(pamo_ctx* c, const double* V, int64_t nv, const int32_t* F, int64_t nf,
                                    int32_t* pairs, int64_t cap, int64_t* npairs) {
  return guarded(c, [&]() -> pamo_status {
    if (!V || !F || !npairs || (cap > 0 && !pairs)) fail(PAMO_ERR_ARG, "null pointer");
    if (nv < 1 || nf < 1 || nf > (int64_t)(INT32_MAX / 3) - 1) fail(PAMO_ERR_ARG, "bad sizes");
    reserve(c, std::max<int64_t>(nv, 4), std::max<int64_t>(nf, 4), Parts{});
    MeshView m;
    m.V = const_cast<double*>(V);
    m.F = const_cast<int*>(F);
    m.twin = nullptr;
    m.vh = nullptr;
    m.flags = nullptr;
    m.nv = (int)nv;
    m.nf = (int)nf;
    fill_i32(c->stream, c->dcnt, C_COUNT, 0);
    hipLaunchKernelGGL(k_check_index, dim3(nblk(3 * nf)), dim3(256), 0, c->stream, F, 3 * nf, (int)nv,
                       c->dcnt + C_ERR);
    check_err_bits(readback(c)[C_ERR]);
    int2* out = pairs ? (int2*)pairs : c->ws.get<int2>("w.pairs", 1);
    *npairs = whole_mesh_pairs(c, m, out, pairs ? cap : 0);
    return PAMO_OK;
  });
}

pamo_status pamo_tri_pairs(pamo_ctx* c, const double* P, const int32_t* ip, const double* Q, const int32_t* iq,
                           int64_t n, uint8_t* out) {
  return guarded(c, [&]() -> pamo_status {
    if (n < 0 || (n > 0 && (!P || !ip || !Q || !iq || !out))) fail(PAMO_ERR_ARG, "bad arguments");
    if (n == 0) return PAMO_OK;
    hipLaunchKernelGGL(k_tri_pairs, dim3(nblk(n, 64)), dim3(64), 0, c->stream, P, ip, Q, iq, n, out);
    PAMO_HIP(hipGetLastError());
    return PAMO_OK;
  });
}

pamo_status pamo_profile_enable(pamo_ctx* c, uint32_t phase_mask) {
  if (!c) return PAMO_ERR_ARG;
  c->prof.mask = phase_mask;
  return PAMO_OK;
}

int32_t pamo_profile_phases(void) { return PH_COUNT; }

const char* pamo_profile_name(int32_t phase) { return phase >= 0 && phase < PH_COUNT ? PH_NAME[phase] : ""; }

pamo_status pamo_profile_read(pamo_ctx* c, int32_t phase, int64_t* launches, double* ms, double* bytes) {
  if (!c || phase < 0 || phase >= PH_COUNT) return PAMO_ERR_ARG;
  return guarded(c, [&]() -> pamo_status {
    PAMO_HIP(hipStreamSynchronize(c->stream));
    prof_resolve(c);
    const auto& a = c->prof.acc[phase];
    if (launches) *launches = a.launches;
    if (ms) *ms = a.ms;
    if (bytes) *bytes = a.bytes;
    return PAMO_OK;
  });
}

pamo_status pamo_profile_reset(pamo_ctx* c) {
  if (!c) return PAMO_ERR_ARG;
  return guarded(c, [&]() -> pamo_status {
    PAMO_HIP(hipStreamSynchronize(c->stream));
    prof_resolve(c);
    for (auto& a : c->prof.acc) a = Prof::Acc();
    return PAMO_OK;
  });
}

}  // extern "C"
