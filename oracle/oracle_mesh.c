/*
 * TEST INFRASTRUCTURE ONLY.  This is the CPU oracle of the parallel
 * intersection-free QEM edge-collapse simplification of PaMO (Sec. 5,
 * "Parallel Intersection-Free Mesh Simplification" algorithm).  Only tests,
 * the smoke check and the benchmark's CPU-baseline leg may call it; the
 * product path never does.
 *
 * It is written to be read against the paper, not to be fast: every round
 * rebuilds its adjacency from the face list, propagates edge costs to
 * triangles in the push form the paper prints (each edge lowers the cost of
 * every triangle of its 1-ring), and runs the check/undo loop as a plain
 * fixed point over all triangles changed by the round.  Faces and vertices
 * are never compacted; dead ones are skipped.  Every id is used only through
 * its order, so a caller that compacts stably sees the same decisions.
 *
 * One round (the numbering is the one the library documentation uses too):
 *   R1  per-vertex quadric: sum, over incident faces in ascending face slot,
 *       of the plane quadric of each face (Garland-Heckbert; Sec. 5.1 "Edge
 *       Cost" names QEM for the Q_ab term of Eq. 1).
 *   R2  placement of the merged vertex: the QEM minimiser when the 3x3 system
 *       is well conditioned and the minimiser lies in the box of the two
 *       closed 1-rings, else the best of midpoint / endpoint / endpoint.
 *       (The paper does not say how it places the vertex.)
 *   R3  edge cost, Eq. 1: Q_ab + w_e l_ab + w_s sum(1 - C_ijk) over the
 *       triangles the collapse generates (summed around the smaller endpoint
 *       first, each star in ascending face slot), w_e = 0.001, w_s = 0.005.
 *   R4  64-bit key: float32 cost mapped to an order-preserving 32-bit code in
 *       the high half, unique edge id in the low half (Sec. 5.1, "Cost
 *       Propagation").  Flagged edges and NaN costs get the largest key.
 *   R5/R6 cost propagation and independent-region selection (Sec. 5.1 and
 *       the figure on independent regions): a triangle takes the minimum key
 *       of every edge whose 1-ring contains it; an edge is collapsed when all
 *       triangles of its 1-ring carry its own key.
 *   R7  local checks on the pre-round mesh: the link condition (Sec. 5.1,
 *       "Edge Collapse"), no generated triangle exactly degenerate, no
 *       generated triangle with a flipped normal.
 *   R8  exact face target: if more collapses pass than are needed, keep the
 *       ones with the smallest keys.
 *   R9  apply all kept collapses at once (their regions are disjoint).
 *   R10 self-intersection test between triangle pairs (Sec. 5.2, Appendix 3).
 *   R11 check/undo fixed point (Sec. 5.3): undo every collapse owning a
 *       triangle of an intersecting pair, repeat until no pair intersects.
 *   R12 commit; invalid-edge flags for the next round and the tolerance
 *       counter (Sec. 5.3, last two paragraphs).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_internal.h"

#define KEY_MAX UINT64_MAX

typedef struct {
    double w_e, w_s;
    int32_t tolerance;
    int32_t max_rounds; /* < 0: no limit */
    double cost_target; /* > 0: collapse only edges whose cost is at most this; the run
                           also ends when a round selects no edge (the target-cost
                           termination the paper offers besides the face count) */
    int32_t prefilter;  /* 1: the link and flip checks (R7) run on every keyed edge before
                           the selection, and failing edges get no key this round, so
                           they do not hold back their neighbourhood (the other order of
                           selection and local checks; the paper applies the link
                           condition during the collapse, Sec. 5.1) */
    int32_t key_mode;   /* 0: R4's float32 key; 1: keys ordered by the float64 cost, then
                           the edge id (the other reading of the cost-to-key conversion
                           of Sec. 5.1, "Cost Propagation"); not with the learned proposal,
                           whose features read the float32 cost from the key */
} oracle_opts;

typedef struct {
    int64_t rounds, commits, candidates, rej_link, rej_flip, rej_isect, capped;
    int64_t undo_hist[5];
    int64_t status; /* 0 target reached, 1 target unreachable, 2 stopped by max_rounds */
} oracle_stats;

typedef struct {
    int64_t faces, verts, edges, candidates, passing, chosen, changed_faces;
    int64_t undo_iters, commits, rej_link, rej_flip, rej_isect, capped;
} oracle_round_log;

typedef struct {
    int64_t nv, nf;
    double *V;
    int32_t *F;
    uint8_t *falive, *valive, *flags;
    int32_t streak;
    /* rebuilt every round */
    int64_t *inc_off;
    int32_t *inc;
    int32_t *twin;
    double *Q;
    uint64_t *key;
} omesh;

static void *xalloc(size_t n) {
    void *p = calloc(n ? n : 1, 1);
    if (!p) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
    return p;
}

/* ------------------------------------------------------------------------ */
/* adjacency                                                                 */
/* ------------------------------------------------------------------------ */

/* incident alive faces of every vertex, in ascending face slot; and the twin
 * (opposite half-edge) of every half-edge h = 3f+c, which runs from F[f][c]
 * to F[f][(c+1)%3].  Returns 0, or -2 when the mesh is not a closed
 * edge-manifold. */
static int build_adjacency(omesh *m) {
    int64_t nv = m->nv, nf = m->nf;
    free(m->inc_off); free(m->inc); free(m->twin);
    m->inc_off = xalloc(sizeof(int64_t) * (size_t)(nv + 1));
    for (int64_t f = 0; f < nf; f++) {
        if (!m->falive[f]) continue;
        for (int c = 0; c < 3; c++) m->inc_off[m->F[3 * f + c] + 1]++;
    }
    for (int64_t v = 0; v < nv; v++) m->inc_off[v + 1] += m->inc_off[v];
    m->inc = xalloc(sizeof(int32_t) * (size_t)(m->inc_off[nv] + 1));
    int64_t *fill = xalloc(sizeof(int64_t) * (size_t)nv);
    for (int64_t f = 0; f < nf; f++) {
        if (!m->falive[f]) continue;
        for (int c = 0; c < 3; c++) {
            int32_t v = m->F[3 * f + c];
            m->inc[m->inc_off[v] + fill[v]++] = (int32_t)f;
        }
    }
    free(fill);
    m->twin = xalloc(sizeof(int32_t) * (size_t)(3 * nf));
    for (int64_t i = 0; i < 3 * nf; i++) m->twin[i] = -1;
    for (int64_t f = 0; f < nf; f++) {
        if (!m->falive[f]) continue;
        for (int c = 0; c < 3; c++) {
            int32_t a = m->F[3 * f + c], b = m->F[3 * f + (c + 1) % 3];
            int found = 0;
            for (int64_t i = m->inc_off[b]; i < m->inc_off[b + 1]; i++) {
                int32_t g = m->inc[i];
                for (int k = 0; k < 3; k++) {
                    if (m->F[3 * g + k] == b && m->F[3 * g + (k + 1) % 3] == a) {
                        if (g == f) continue;
                        m->twin[3 * f + c] = 3 * g + k;
                        found++;
                    }
                }
            }
            if (found != 1) return -2;
        }
    }
    return 0;
}

static int face_has(const omesh *m, int32_t f, int32_t v) {
    const int32_t *t = m->F + 3 * (int64_t)f;
    return t[0] == v || t[1] == v || t[2] == v;
}

/* faces of star(a) u star(b), ascending, each once */
static int ring_faces(const omesh *m, int32_t a, int32_t b, int32_t *out, int cap) {
    int64_t i = m->inc_off[a], ie = m->inc_off[a + 1];
    int64_t j = m->inc_off[b], je = m->inc_off[b + 1];
    int n = 0;
    while (i < ie || j < je) {
        int32_t fa = i < ie ? m->inc[i] : INT32_MAX;
        int32_t fb = j < je ? m->inc[j] : INT32_MAX;
        int32_t f;
        if (fa < fb) { f = fa; i++; }
        else if (fb < fa) { f = fb; j++; }
        else { f = fa; i++; j++; }
        if (n >= cap) return -1;
        out[n++] = f;
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* quadrics (R1)                                                             */
/* ------------------------------------------------------------------------ */

/* plane quadric of one face: unit normal n of (p1-p0)x(p2-p0), offset
 * d = -n.p0, K = [n;d][n;d]^T stored as its 10 upper-triangle entries
 * (xx, xy, xz, xw, yy, yz, yw, zz, zw, ww). */
static void face_quadric(const double *p0, const double *p1, const double *p2, double *K) {
    double e1x = p1[0] - p0[0], e1y = p1[1] - p0[1], e1z = p1[2] - p0[2];
    double e2x = p2[0] - p0[0], e2y = p2[1] - p0[1], e2z = p2[2] - p0[2];
    double nx = e1y * e2z - e1z * e2y;
    double ny = e1z * e2x - e1x * e2z;
    double nz = e1x * e2y - e1y * e2x;
    double len = sqrt(nx * nx + ny * ny + nz * nz);
    nx = nx / len;
    ny = ny / len;
    nz = nz / len;
    double d = -(nx * p0[0] + ny * p0[1] + nz * p0[2]);
    K[0] = nx * nx; K[1] = nx * ny; K[2] = nx * nz; K[3] = nx * d;
    K[4] = ny * ny; K[5] = ny * nz; K[6] = ny * d;
    K[7] = nz * nz; K[8] = nz * d;
    K[9] = d * d;
}

static void compute_quadrics(omesh *m) {
    free(m->Q);
    m->Q = xalloc(sizeof(double) * 10 * (size_t)m->nv);
    double K[10];
    for (int64_t f = 0; f < m->nf; f++) {
        if (!m->falive[f]) continue;
        const int32_t *t = m->F + 3 * f;
        face_quadric(m->V + 3 * (int64_t)t[0], m->V + 3 * (int64_t)t[1], m->V + 3 * (int64_t)t[2], K);
        for (int c = 0; c < 3; c++) {
            double *q = m->Q + 10 * (int64_t)t[c];
            for (int i = 0; i < 10; i++) q[i] = q[i] + K[i];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* placement and cost (R2, R3)                                               */
/* ------------------------------------------------------------------------ */

/* v^T Q v with v = (x, y, z, 1) */
static double quadric_eval(const double *q, const double *v) {
    double x = v[0], y = v[1], z = v[2];
    double qx = q[0] * x + q[1] * y + q[2] * z + q[3];
    double qy = q[1] * x + q[4] * y + q[5] * z + q[6];
    double qz = q[2] * x + q[5] * y + q[7] * z + q[8];
    double qw = q[3] * x + q[6] * y + q[8] * z + q[9];
    return qx * x + qy * y + qz * z + qw;
}

/* edge (s, r) with s < r; ring = faces of star(s) u star(r), ascending */
static void placement(const omesh *m, int32_t s, int32_t r, const int32_t *ring, int nring,
                      const double *q, double *vbar) {
    double a00 = q[0], a01 = q[1], a02 = q[2], a11 = q[4], a12 = q[5], a22 = q[7];
    double r0 = -q[3], r1 = -q[6], r2 = -q[8];
    double c00 = a11 * a22 - a12 * a12;
    double c01 = a01 * a22 - a12 * a02;
    double c02 = a01 * a12 - a11 * a02;
    double det = a00 * c00 - a01 * c01 + a02 * c02;
    double tr3 = (a00 + a11 + a22) / 3.0;
    double thr = 1e-10 * (tr3 * tr3 * tr3);
    if (fabs(det) > thr) {
        /* Cramer's rule for A v = -b */
        double dx = r0 * c00 - a01 * (r1 * a22 - a12 * r2) + a02 * (r1 * a12 - a11 * r2);
        double dy = a00 * (r1 * a22 - a12 * r2) - r0 * c01 + a02 * (a01 * r2 - r1 * a02);
        double dz = a00 * (a11 * r2 - r1 * a12) - a01 * (a01 * r2 - r1 * a02) + r0 * c02;
        double v[3] = {dx / det, dy / det, dz / det};
        /* box of the closed 1-rings of both endpoints */
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int i = 0; i < nring; i++) {
            const int32_t *t = m->F + 3 * (int64_t)ring[i];
            for (int c = 0; c < 3; c++) {
                const double *p = m->V + 3 * (int64_t)t[c];
                for (int k = 0; k < 3; k++) {
                    if (p[k] < lo[k]) lo[k] = p[k];
                    if (p[k] > hi[k]) hi[k] = p[k];
                }
            }
        }
        int inside = 1;
        for (int k = 0; k < 3; k++)
            if (!(v[k] >= lo[k] && v[k] <= hi[k])) inside = 0;
        if (inside) {
            vbar[0] = v[0]; vbar[1] = v[1]; vbar[2] = v[2];
            return;
        }
    }
    const double *ps = m->V + 3 * (int64_t)s, *pr = m->V + 3 * (int64_t)r;
    double mid[3] = {(ps[0] + pr[0]) * 0.5, (ps[1] + pr[1]) * 0.5, (ps[2] + pr[2]) * 0.5};
    const double *best = mid;
    double qb = quadric_eval(q, mid);
    double qs = quadric_eval(q, ps);
    if (qs < qb) { best = ps; qb = qs; }
    double qr = quadric_eval(q, pr);
    if (qr < qb) { best = pr; qb = qr; }
    vbar[0] = best[0]; vbar[1] = best[1]; vbar[2] = best[2];
}

/* corner position of face f after collapsing (s, r) onto vbar */
static const double *corner_after(const omesh *m, int32_t f, int c, int32_t s, int32_t r, const double *vbar) {
    int32_t v = m->F[3 * (int64_t)f + c];
    return (v == s || v == r) ? vbar : m->V + 3 * (int64_t)v;
}

static const double SKINNY_K = 3.4641016151377544; /* 2 sqrt(3), so 4 sqrt(3) A = SKINNY_K |n| */

/* 1 - C_ijk for the triangle p0 p1 p2 (Eq. 1) */
static double skinny_term(const double *p0, const double *p1, const double *p2) {
    double e1x = p1[0] - p0[0], e1y = p1[1] - p0[1], e1z = p1[2] - p0[2];
    double e2x = p2[0] - p0[0], e2y = p2[1] - p0[1], e2z = p2[2] - p0[2];
    double e3x = p2[0] - p1[0], e3y = p2[1] - p1[1], e3z = p2[2] - p1[2];
    double nx = e1y * e2z - e1z * e2y;
    double ny = e1z * e2x - e1x * e2z;
    double nz = e1x * e2y - e1y * e2x;
    double nn = sqrt(nx * nx + ny * ny + nz * nz);
    double l01 = e1x * e1x + e1y * e1y + e1z * e1z;
    double l12 = e3x * e3x + e3y * e3y + e3z * e3z;
    double l20 = e2x * e2x + e2y * e2y + e2z * e2z;
    double lsum = l01 + l12 + l20;
    return 1.0 - (SKINNY_K * nn) / lsum;
}

#define RING_CAP 4096

/* cost of the edge (a, b) and its placement (R2, R3) */
static double edge_cost(const omesh *m, int32_t a, int32_t b, double w_e, double w_s, double *vbar) {
    int32_t s = a < b ? a : b, r = a < b ? b : a;
    int32_t ring[RING_CAP];
    int nring = ring_faces(m, s, r, ring, RING_CAP);
    if (nring < 0) { fprintf(stderr, "oracle: ring too large\n"); abort(); }
    double q[10];
    const double *qs = m->Q + 10 * (int64_t)s, *qr = m->Q + 10 * (int64_t)r;
    for (int i = 0; i < 10; i++) q[i] = qs[i] + qr[i];
    placement(m, s, r, ring, nring, q, vbar);
    const double *ps = m->V + 3 * (int64_t)s, *pr = m->V + 3 * (int64_t)r;
    double dx = ps[0] - pr[0], dy = ps[1] - pr[1], dz = ps[2] - pr[2];
    double lab = sqrt(dx * dx + dy * dy + dz * dz);
    /* The sum over the generated triangles has no order in the paper; it runs
     * over the faces around s in ascending slot, then those around r.  The two
     * faces holding both s and r are removed by the collapse and skipped, so
     * every generated triangle is counted once. */
    double S = 0.0;
    for (int side = 0; side < 2; side++) {
        int32_t v = side ? r : s;
        for (int64_t i = m->inc_off[v]; i < m->inc_off[v + 1]; i++) {
            int32_t f = m->inc[i];
            if (face_has(m, f, s) && face_has(m, f, r)) continue;
            S = S + skinny_term(corner_after(m, f, 0, s, r, vbar), corner_after(m, f, 1, s, r, vbar),
                                corner_after(m, f, 2, s, r, vbar));
        }
    }
    return quadric_eval(q, vbar) + w_e * lab + w_s * S;
}

/* R4: order-preserving 32-bit code of a float32 cost, unique id below */
static uint64_t make_key(double cost, uint32_t edge_id) {
    if (cost != cost) return KEY_MAX;
    float c32 = (float)cost;
    uint32_t u;
    memcpy(&u, &c32, 4);
    uint32_t o = (u >> 31) ? ~u : (u | 0x80000000u);
    return ((uint64_t)o << 32) | edge_id;
}

/* key_mode 1: a total order code of a float64 cost (zero of either sign as
 * +0, so equal costs get equal codes) */
static uint64_t ord64(double c) {
    if (c == 0.0) c = 0.0;
    uint64_t u;
    memcpy(&u, &c, 8);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

static const uint64_t *g_codes; /* qsort helper (single-threaded oracle) */
static int cmp_code_then_id(const void *x, const void *y) {
    int64_t a = *(const int64_t *)x, b = *(const int64_t *)y;
    if (g_codes[a] != g_codes[b]) return g_codes[a] < g_codes[b] ? -1 : 1;
    return (a > b) - (a < b);
}

static int edge_flagged(const omesh *m, int64_t h) {
    return m->flags[h] || m->flags[m->twin[h]];
}

/* keys at every half-edge that represents its edge (h < twin(h)); KEY_MAX
 * elsewhere, and for edges costing more than cost_target when it is > 0.
 * key_mode 1: keys are only ever compared, so each keyed edge takes as key its
 * rank in the order of (float64 cost, edge id) */
static void compute_keys_capped(omesh *m, double w_e, double w_s, double cost_target, int key_mode) {
    free(m->key);
    int64_t nh = 3 * m->nf;
    m->key = xalloc(sizeof(uint64_t) * (size_t)nh);
    uint64_t *code = key_mode ? xalloc(sizeof(uint64_t) * (size_t)nh) : NULL;
    int64_t *keyed = key_mode ? xalloc(sizeof(int64_t) * (size_t)(nh + 1)) : NULL;
    int64_t nk = 0;
    for (int64_t h = 0; h < nh; h++) {
        m->key[h] = KEY_MAX;
        if (!m->falive[h / 3] || m->twin[h] < h) continue;
        if (edge_flagged(m, h)) continue;
        int32_t a = m->F[h], b = m->F[3 * (h / 3) + (h % 3 + 1) % 3];
        double vbar[3];
        double cost = edge_cost(m, a, b, w_e, w_s, vbar);
        if (cost_target > 0 && cost > cost_target) continue;
        if (!key_mode) {
            m->key[h] = make_key(cost, (uint32_t)h);
        } else if (cost == cost) {
            code[h] = ord64(cost);
            keyed[nk++] = h;
        }
    }
    if (key_mode) {
        g_codes = code;
        qsort(keyed, (size_t)nk, sizeof(int64_t), cmp_code_then_id);
        for (int64_t i = 0; i < nk; i++) m->key[keyed[i]] = (uint64_t)i;
        free(code);
        free(keyed);
    }
}

static void compute_keys(omesh *m, double w_e, double w_s) { compute_keys_capped(m, w_e, w_s, 0.0, 0); }

/* R5/R6 in the push form of the paper: C_t = min over edges e whose 1-ring
 * contains t of C_e; e is chosen when C_t = C_e for every t of its 1-ring. */
static int64_t select_edges(const omesh *m, int32_t *cand) {
    uint64_t *Ct = xalloc(sizeof(uint64_t) * (size_t)m->nf);
    for (int64_t f = 0; f < m->nf; f++) Ct[f] = KEY_MAX;
    int32_t ring[RING_CAP];
    for (int64_t h = 0; h < 3 * m->nf; h++) {
        uint64_t k = m->key[h];
        if (k == KEY_MAX) continue;
        int32_t a = m->F[h], b = m->F[3 * (h / 3) + (h % 3 + 1) % 3];
        int n = ring_faces(m, a, b, ring, RING_CAP);
        for (int i = 0; i < n; i++)
            if (k < Ct[ring[i]]) Ct[ring[i]] = k;
    }
    int64_t nc = 0;
    for (int64_t h = 0; h < 3 * m->nf; h++) {
        uint64_t k = m->key[h];
        if (k == KEY_MAX) continue;
        int32_t a = m->F[h], b = m->F[3 * (h / 3) + (h % 3 + 1) % 3];
        int n = ring_faces(m, a, b, ring, RING_CAP);
        int all = 1;
        for (int i = 0; i < n; i++)
            if (Ct[ring[i]] != k) { all = 0; break; }
        if (all) cand[nc++] = (int32_t)h;
    }
    free(Ct);
    return nc;
}

/* ------------------------------------------------------------------------ */
/* local checks (R7)                                                         */
/* ------------------------------------------------------------------------ */

static int cmp_i32(const void *x, const void *y) {
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}
static int cmp_i64(const void *x, const void *y) {
    int64_t a = *(const int64_t *)x, b = *(const int64_t *)y;
    return (a > b) - (a < b);
}

/* link of v: vertex set and edge set (edges as lo*2^32+hi) */
static void link_of(const omesh *m, int32_t v, int32_t *lv, int *nlv, int64_t *le, int *nle) {
    *nlv = 0;
    *nle = 0;
    for (int64_t i = m->inc_off[v]; i < m->inc_off[v + 1]; i++) {
        const int32_t *t = m->F + 3 * (int64_t)m->inc[i];
        int32_t o[2], k = 0;
        for (int c = 0; c < 3; c++)
            if (t[c] != v) o[k++] = t[c];
        lv[(*nlv)++] = o[0];
        lv[(*nlv)++] = o[1];
        int32_t lo = o[0] < o[1] ? o[0] : o[1], hi = o[0] < o[1] ? o[1] : o[0];
        le[(*nle)++] = ((int64_t)lo << 32) | (int64_t)hi;
    }
    qsort(lv, (size_t)*nlv, sizeof(int32_t), cmp_i32);
    int u = 0;
    for (int i = 0; i < *nlv; i++)
        if (i == 0 || lv[i] != lv[i - 1]) lv[u++] = lv[i];
    *nlv = u;
    qsort(le, (size_t)*nle, sizeof(int64_t), cmp_i64);
}

/* link condition Lk(a) n Lk(b) = Lk(ab) (Dey et al.), compared as sets */
static int link_ok(const omesh *m, int32_t a, int32_t b) {
    static int32_t la[RING_CAP], lb[RING_CAP], lab[RING_CAP];
    static int64_t ea[RING_CAP], eb[RING_CAP];
    int nla, nlb, nea, neb;
    link_of(m, a, la, &nla, ea, &nea);
    link_of(m, b, lb, &nlb, eb, &neb);
    /* Lk(ab): third vertex of every face containing both a and b */
    int nlab = 0;
    for (int64_t i = m->inc_off[a]; i < m->inc_off[a + 1]; i++) {
        int32_t f = m->inc[i];
        if (!face_has(m, f, b)) continue;
        for (int c = 0; c < 3; c++) {
            int32_t v = m->F[3 * (int64_t)f + c];
            if (v != a && v != b) lab[nlab++] = v;
        }
    }
    qsort(lab, (size_t)nlab, sizeof(int32_t), cmp_i32);
    /* vertex part of the intersection */
    int32_t inter[RING_CAP];
    int ni = 0;
    for (int i = 0, j = 0; i < nla && j < nlb;) {
        if (la[i] < lb[j]) i++;
        else if (lb[j] < la[i]) j++;
        else { inter[ni++] = la[i]; i++; j++; }
    }
    if (ni != nlab) return 0;
    for (int i = 0; i < ni; i++)
        if (inter[i] != lab[i]) return 0;
    /* edge part: Lk(ab) has no edges */
    for (int i = 0, j = 0; i < nea && j < neb;) {
        if (ea[i] < eb[j]) i++;
        else if (eb[j] < ea[i]) j++;
        else return 0;
    }
    return 1;
}

/* reason: 0 pass, 1 link, 2 degenerate or flipped generated triangle */
static int local_check(const omesh *m, int32_t a, int32_t b, const double *vbar) {
    if (!link_ok(m, a, b)) return 1;
    int32_t s = a < b ? a : b, r = a < b ? b : a;
    int32_t ring[RING_CAP];
    int n = ring_faces(m, s, r, ring, RING_CAP);
    for (int i = 0; i < n; i++) {
        int32_t f = ring[i];
        if (face_has(m, f, s) && face_has(m, f, r)) continue;
        const double *p0 = corner_after(m, f, 0, s, r, vbar);
        const double *p1 = corner_after(m, f, 1, s, r, vbar);
        const double *p2 = corner_after(m, f, 2, s, r, vbar);
        if (o_degenerate(p0, p1, p2)) return 2;
        const int32_t *t = m->F + 3 * (int64_t)f;
        const double *o0 = m->V + 3 * (int64_t)t[0], *o1 = m->V + 3 * (int64_t)t[1], *o2 = m->V + 3 * (int64_t)t[2];
        double ax = o1[0] - o0[0], ay = o1[1] - o0[1], az = o1[2] - o0[2];
        double bx = o2[0] - o0[0], by = o2[1] - o0[1], bz = o2[2] - o0[2];
        double nox = ay * bz - az * by, noy = az * bx - ax * bz, noz = ax * by - ay * bx;
        double cx = p1[0] - p0[0], cy = p1[1] - p0[1], cz = p1[2] - p0[2];
        double dx = p2[0] - p0[0], dy = p2[1] - p0[1], dz = p2[2] - p0[2];
        double nnx = cy * dz - cz * dy, nny = cz * dx - cx * dz, nnz = cx * dy - cy * dx;
        double dot = nox * nnx + noy * nny + noz * nnz;
        if (!(dot > 0.0)) return 2;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* self-intersection search (R10, R11)                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
    int g[3];
    double lo[3], h[3];
    int64_t *off;
    int32_t *items;
} ogrid;

static void face_box(const omesh *m, int64_t f, double *lo, double *hi) {
    const int32_t *t = m->F + 3 * f;
    for (int k = 0; k < 3; k++) { lo[k] = INFINITY; hi[k] = -INFINITY; }
    for (int c = 0; c < 3; c++) {
        const double *p = m->V + 3 * (int64_t)t[c];
        for (int k = 0; k < 3; k++) {
            if (p[k] < lo[k]) lo[k] = p[k];
            if (p[k] > hi[k]) hi[k] = p[k];
        }
    }
}

static int cell_of(const ogrid *G, int k, double x) {
    double t = (x - G->lo[k]) / G->h[k];
    int i = (int)floor(t);
    if (i < 0) i = 0;
    if (i >= G->g[k]) i = G->g[k] - 1;
    return i;
}

/* uniform grid over the boxes of all alive faces: a face is listed in every
 * cell its box touches.  It only prunes pairs whose boxes are disjoint. */
static void grid_build(const omesh *m, ogrid *G) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int64_t nalive = 0;
    for (int64_t f = 0; f < m->nf; f++) {
        if (!m->falive[f]) continue;
        nalive++;
        double a[3], b[3];
        face_box(m, f, a, b);
        for (int k = 0; k < 3; k++) {
            if (a[k] < lo[k]) lo[k] = a[k];
            if (b[k] > hi[k]) hi[k] = b[k];
        }
    }
    int g = (int)cbrt((double)nalive / 2.0);
    if (g < 1) g = 1;
    if (g > 512) g = 512;
    for (int k = 0; k < 3; k++) {
        G->g[k] = g;
        G->lo[k] = lo[k];
        G->h[k] = (hi[k] - lo[k]) / g;
        if (!(G->h[k] > 0)) G->h[k] = 1.0;
    }
    int64_t ncell = (int64_t)g * g * g;
    G->off = xalloc(sizeof(int64_t) * (size_t)(ncell + 1));
    for (int pass = 0; pass < 2; pass++) {
        int64_t *fill = pass ? xalloc(sizeof(int64_t) * (size_t)ncell) : NULL;
        for (int64_t f = 0; f < m->nf; f++) {
            if (!m->falive[f]) continue;
            double a[3], b[3];
            face_box(m, f, a, b);
            int i0 = cell_of(G, 0, a[0]), i1 = cell_of(G, 0, b[0]);
            int j0 = cell_of(G, 1, a[1]), j1 = cell_of(G, 1, b[1]);
            int k0 = cell_of(G, 2, a[2]), k1 = cell_of(G, 2, b[2]);
            for (int i = i0; i <= i1; i++)
                for (int j = j0; j <= j1; j++)
                    for (int k = k0; k <= k1; k++) {
                        int64_t c = ((int64_t)i * g + j) * g + k;
                        if (!pass) G->off[c + 1]++;
                        else G->items[G->off[c] + fill[c]++] = (int32_t)f;
                    }
        }
        if (!pass) {
            for (int64_t c = 0; c < ncell; c++) G->off[c + 1] += G->off[c];
            G->items = xalloc(sizeof(int32_t) * (size_t)(G->off[ncell] + 1));
        } else {
            free(fill);
        }
    }
}

static void grid_free(ogrid *G) {
    free(G->off);
    free(G->items);
}

static int boxes_overlap(const double *alo, const double *ahi, const double *blo, const double *bhi) {
    for (int k = 0; k < 3; k++)
        if (ahi[k] < blo[k] || bhi[k] < alo[k]) return 0;
    return 1;
}

static int pair_intersects(const omesh *m, int64_t t, int64_t u) {
    const int32_t *a = m->F + 3 * t, *b = m->F + 3 * u;
    const double *P[3] = {m->V + 3 * (int64_t)a[0], m->V + 3 * (int64_t)a[1], m->V + 3 * (int64_t)a[2]};
    const double *Q[3] = {m->V + 3 * (int64_t)b[0], m->V + 3 * (int64_t)b[1], m->V + 3 * (int64_t)b[2]};
    return o_tri_pair(P, a, Q, b);
}

/* calls visit(ctx, t, u) for every alive face u != t whose box meets t's box
 * and that forms an intersecting pair with t */
typedef void (*pair_visit)(void *ctx, int64_t t, int64_t u);

static void query_face(const omesh *m, const ogrid *G, int64_t t, int64_t *stamp, int64_t stamp_id,
                       pair_visit visit, void *ctx) {
    double a[3], b[3];
    face_box(m, t, a, b);
    int i0 = cell_of(G, 0, a[0]), i1 = cell_of(G, 0, b[0]);
    int j0 = cell_of(G, 1, a[1]), j1 = cell_of(G, 1, b[1]);
    int k0 = cell_of(G, 2, a[2]), k1 = cell_of(G, 2, b[2]);
    int g = G->g[0];
    for (int i = i0; i <= i1; i++)
        for (int j = j0; j <= j1; j++)
            for (int k = k0; k <= k1; k++) {
                int64_t c = ((int64_t)i * g + j) * g + k;
                for (int64_t e = G->off[c]; e < G->off[c + 1]; e++) {
                    int64_t u = G->items[e];
                    if (u == t || stamp[u] == stamp_id) continue;
                    stamp[u] = stamp_id;
                    double c0[3], c1[3];
                    face_box(m, u, c0, c1);
                    if (!boxes_overlap(a, b, c0, c1)) continue;
                    if (pair_intersects(m, t, u)) visit(ctx, t, u);
                }
            }
}

/* ------------------------------------------------------------------------ */
/* learned proposal (an addition to the method; the paper has no network)    */
/* ------------------------------------------------------------------------ */
/* A small network scores every selected candidate before its checks.  The
 * ones it scores below a threshold are set aside for the round (their key
 * becomes the largest) and the selection is redone, so that a neighbour of a
 * likely rejection can be collapsed instead.  Every collapse still passes
 * every check; a round that sets candidates aside and then commits nothing is
 * run again without the network.  The network is consulted only in rounds
 * that follow a round whose checks rejected at least one candidate (the first
 * round is plain): where nothing gets rejected it has nothing to predict.
 *
 * Per-face state for the overlap feature: ovl[f] counts the alive faces that
 * share no vertex with f and whose float64 boxes meet f's box (closed).  It is
 * counted on the whole input, and again for each face a round changes, on the
 * tentative mesh of that round's first check, kept when the face's collapse
 * is committed. */

#define NF_USED 11
#define NFEAT 32

typedef struct {
    float w1[64][32]; float b1[64];   /* w1[j][k]: input k -> unit j */
    float w2[64][64]; float b2[64];
    float w3[64];     float b3;
    int32_t e1, e2, e3;               /* weight grids 2^-e (checked by the library, unused here) */
    int32_t a1, a2;                   /* activation shifts */
    float threshold;                  /* set aside when logit < threshold */
} oracle_mlp;

/* power-of-two scale of each feature before rounding to an integer in
 * [-127, 127] */
static const int FEAT_SHIFT[NF_USED] = {2, 3, 7, 7, 6, 6, 2, 2, 4, 0, 2};

/* piecewise-linear log2: exact at powers of two, linear in between */
static double plog2(double c) {
    if (!(c > 0.0)) return -64.0;
    if (isinf(c)) return 64.0;
    int e;
    double mant = frexp(c, &e); /* c = mant 2^e, mant in [0.5, 1) */
    return (double)(e - 1) + (2.0 * mant - 1.0);
}

static float quantize_feature(double f, int shift) {
    double q = rint(ldexp(f, shift));
    if (q != q) return 0.0f;
    if (q > 127.0) q = 127.0;
    if (q < -127.0) q = -127.0;
    return (float)q;
}

static double seg_len(const double *p, const double *q) {
    double dx = q[0] - p[0], dy = q[1] - p[1], dz = q[2] - p[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

/* unnormalised normal (p1 - p0) x (p2 - p0) of face f, corners in slot order */
static void face_normal(const omesh *m, int64_t f, double *n) {
    const double *p0 = m->V + 3 * (int64_t)m->F[3 * f];
    const double *p1 = m->V + 3 * (int64_t)m->F[3 * f + 1];
    const double *p2 = m->V + 3 * (int64_t)m->F[3 * f + 2];
    double e1x = p1[0] - p0[0], e1y = p1[1] - p0[1], e1z = p1[2] - p0[2];
    double e2x = p2[0] - p0[0], e2y = p2[1] - p0[1], e2z = p2[2] - p0[2];
    n[0] = e1y * e2z - e1z * e2y;
    n[1] = e1z * e2x - e1x * e2z;
    n[2] = e1x * e2y - e1y * e2x;
}

/* cosine of the angle between two normals (1 when either is zero) */
static double normal_cos(const double *n0, const double *n1) {
    double d = n0[0] * n1[0] + n0[1] * n1[1] + n0[2] * n1[2];
    double q = (n0[0] * n0[0] + n0[1] * n0[1] + n0[2] * n0[2]) * (n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2]);
    if (!(q > 0.0)) return 1.0;
    return d / sqrt(q);
}

/* cosine of the angle between the normals of the two faces at the edge of
 * half-edge h (1 where the surface is flat there) */
static double edge_cos(const omesh *m, int64_t h) {
    double n0[3], n1[3];
    face_normal(m, h / 3, n0);
    face_normal(m, m->twin[h] / 3, n1);
    return normal_cos(n0, n1);
}

/* cost of an edge as its key stores it (float32, widened) */
static double key_cost(uint64_t key) {
    uint32_t k = (uint32_t)(key >> 32);
    uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    float f;
    memcpy(&f, &u, sizeof f);
    return (double)f;
}

/* The features of the edge of half-edge h, quantised (NFEAT values, the
 * unused ones zero).  S = star(a) u star(b), spokes = edges of S's faces that
 * contain a or b.
 *   0 plog2 of the edge cost (Eq. 1)            1 plog2 of the edge length
 *   2 length / longest spoke                    3 shortest spoke / length
 *   4 cos of the angle between the normals of the edge's two faces (1: flat)
 *   5 smallest such cos over the spokes
 *   6 valence of a   7 valence of b             8 common neighbours of a and b
 *   9 sum of ovl over S                         10 largest ovl over S */
static void edge_features(const omesh *m, const int32_t *ovl, int64_t h, float *x) {
    int32_t a = m->F[h], b = m->F[3 * (h / 3) + (h % 3 + 1) % 3];
    double f[NF_USED];
    int32_t ring[RING_CAP];
    int n = ring_faces(m, a, b, ring, RING_CAP);
    double le = seg_len(m->V + 3 * (int64_t)a, m->V + 3 * (int64_t)b);
    double lmax = 0.0, lmin = INFINITY, cmin = INFINITY;
    int64_t osum = 0, omax = 0;
    for (int i = 0; i < n; i++) {
        int64_t g = ring[i];
        for (int c = 0; c < 3; c++) {
            int32_t u = m->F[3 * g + c], w = m->F[3 * g + (c + 1) % 3];
            if (u != a && u != b && w != a && w != b) continue;
            double l = seg_len(m->V + 3 * (int64_t)u, m->V + 3 * (int64_t)w);
            if (l > lmax) lmax = l;
            if (l < lmin) lmin = l;
            double cs = edge_cos(m, 3 * g + c);
            if (cs < cmin) cmin = cs;
        }
        int64_t o = ovl ? ovl[g] : 0;
        osum += o;
        if (o > omax) omax = o;
    }
    /* common neighbours: vertices other than a, b on faces of both stars */
    int common = 0;
    for (int64_t i = m->inc_off[a]; i < m->inc_off[a + 1]; i++) {
        int32_t g = m->inc[i];
        for (int c = 0; c < 3; c++) {
            int32_t v = m->F[3 * (int64_t)g + c];
            if (v == a || v == b) continue;
            /* count v once: only from the first face of star(a) holding it */
            int first = 1;
            for (int64_t j = m->inc_off[a]; j < i && first; j++)
                if (face_has(m, m->inc[j], v)) first = 0;
            if (!first) continue;
            int inb = 0;
            for (int64_t j = m->inc_off[b]; j < m->inc_off[b + 1] && !inb; j++)
                if (face_has(m, m->inc[j], v)) inb = 1;
            common += inb;
        }
    }
    f[0] = plog2(key_cost(m->key[h]));
    f[1] = plog2(le);
    f[2] = le / lmax;
    f[3] = lmin / le;
    f[4] = edge_cos(m, h);
    f[5] = cmin;
    f[6] = (double)(m->inc_off[a + 1] - m->inc_off[a]);
    f[7] = (double)(m->inc_off[b + 1] - m->inc_off[b]);
    f[8] = (double)common;
    f[9] = (double)osum;
    f[10] = (double)omax;
    for (int k = 0; k < NFEAT; k++) x[k] = k < NF_USED ? quantize_feature(f[k], FEAT_SHIFT[k]) : 0.0f;
}

/* the network on one quantised feature vector: 32 -> 64 -> 64 -> 1, ReLU,
 * each hidden activation scaled by 2^a and rounded to an integer in [0, 127].
 * Weights lie on grids fine enough and sums are short enough that every
 * float64 operation here is exact. */
static double mlp_logit(const oracle_mlp *M, const float *x) {
    double h1[64], h2[64];
    for (int j = 0; j < 64; j++) {
        double acc = M->b1[j];
        for (int k = 0; k < 32; k++) acc += (double)M->w1[j][k] * (double)x[k];
        if (acc < 0.0) acc = 0.0;
        double q = rint(ldexp(acc, M->a1));
        h1[j] = q > 127.0 ? 127.0 : q;
    }
    for (int j = 0; j < 64; j++) {
        double acc = M->b2[j];
        for (int k = 0; k < 64; k++) acc += (double)M->w2[j][k] * h1[k];
        if (acc < 0.0) acc = 0.0;
        double q = rint(ldexp(acc, M->a2));
        h2[j] = q > 127.0 ? 127.0 : q;
    }
    double acc = M->b3;
    for (int k = 0; k < 64; k++) acc += (double)M->w3[k] * h2[k];
    return acc;
}

/* ovl of face t on the current mesh (t alive) */
static int32_t overlap_count(const omesh *m, const ogrid *G, int64_t t, int64_t *stamp, int64_t stamp_id) {
    double a[3], b[3];
    face_box(m, t, a, b);
    int i0 = cell_of(G, 0, a[0]), i1 = cell_of(G, 0, b[0]);
    int j0 = cell_of(G, 1, a[1]), j1 = cell_of(G, 1, b[1]);
    int k0 = cell_of(G, 2, a[2]), k1 = cell_of(G, 2, b[2]);
    int g = G->g[0];
    int32_t n = 0;
    for (int i = i0; i <= i1; i++)
        for (int j = j0; j <= j1; j++)
            for (int k = k0; k <= k1; k++) {
                int64_t c = ((int64_t)i * g + j) * g + k;
                for (int64_t e = G->off[c]; e < G->off[c + 1]; e++) {
                    int64_t u = G->items[e];
                    if (u == t || stamp[u] == stamp_id) continue;
                    stamp[u] = stamp_id;
                    double c0[3], c1[3];
                    face_box(m, u, c0, c1);
                    if (!boxes_overlap(a, b, c0, c1)) continue;
                    const int32_t *tu = m->F + 3 * u;
                    if (face_has(m, (int32_t)t, tu[0]) || face_has(m, (int32_t)t, tu[1]) ||
                        face_has(m, (int32_t)t, tu[2]))
                        continue;
                    n++;
                }
            }
    return n;
}

/* ovl of every alive face */
static void overlap_init(const omesh *m, int32_t *ovl) {
    ogrid G;
    grid_build(m, &G);
    int64_t *stamp = xalloc(sizeof(int64_t) * (size_t)m->nf);
    for (int64_t f = 0; f < m->nf; f++) stamp[f] = -1;
    for (int64_t f = 0; f < m->nf; f++) ovl[f] = m->falive[f] ? overlap_count(m, &G, f, stamp, f) : 0;
    free(stamp);
    grid_free(&G);
}

/* ------------------------------------------------------------------------ */
/* one round                                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t ncand;
    int32_t *cand;     /* representative half-edge of each candidate, ascending */
    uint8_t *reason;   /* 0 committed, 1 link, 2 flip/degenerate, 3 intersection, 4 capped */
    double *vbar;      /* 3 per candidate */
    int64_t passing, chosen, changed, undo_iters, commits;
    int64_t demoted;   /* learned mode: candidates set aside by the network */
    int retry;         /* learned mode: nothing committed with set-aside candidates; rerun plain */
} round_out;

typedef struct {
    const omesh *m;
    const int32_t *owner;
    const uint8_t *applied;
    uint8_t *mark;
    int64_t nmark;
} undo_ctx;

static void mark_owners(void *vctx, int64_t t, int64_t u) {
    undo_ctx *c = vctx;
    int32_t ot = c->owner[t], ou = c->owner[u];
    if (ot >= 0 && c->applied[ot] && !c->mark[ot]) { c->mark[ot] = 1; c->nmark++; }
    if (ou >= 0 && c->applied[ou] && !c->mark[ou]) { c->mark[ou] = 1; c->nmark++; }
}

static const uint64_t *g_sort_keys; /* qsort helper (single-threaded oracle) */
static int cmp_by_key(const void *x, const void *y) {
    uint64_t a = g_sort_keys[*(const int32_t *)x], b = g_sort_keys[*(const int32_t *)y];
    return (a > b) - (a < b);
}

static int64_t count_alive_faces(const omesh *m) {
    int64_t n = 0;
    for (int64_t f = 0; f < m->nf; f++) n += m->falive[f];
    return n;
}

/* one full round; returns 0 or a negative error */
/* mlp (may be NULL): the learned proposal; ovl (may be NULL): per-face
 * overlap counts, kept up to date when given */
static int run_round(omesh *m, int64_t target_eff, const oracle_opts *opt, round_out *out,
                     int stop_after_check, const oracle_mlp *mlp, int32_t *ovl) {
    int err = build_adjacency(m);
    if (err) return err;
    compute_quadrics(m);
    compute_keys_capped(m, opt->w_e, opt->w_s, opt->cost_target, opt->key_mode);
    int64_t nf = m->nf, nv = m->nv;
    if (opt->prefilter) {
        /* R7 on every keyed edge, on the pre-round mesh: a failing edge is
           not selectable this round (and is not flagged: it was never a
           candidate) */
        double vb[3];
        for (int64_t h = 0; h < 3 * nf; h++) {
            if (m->key[h] == KEY_MAX) continue;
            int32_t a = m->F[h], b = m->F[3 * (h / 3) + (h % 3 + 1) % 3];
            (void)edge_cost(m, a, b, opt->w_e, opt->w_s, vb);
            if (local_check(m, a, b, vb) != 0) m->key[h] = KEY_MAX;
        }
    }

    int32_t *cand = xalloc(sizeof(int32_t) * (size_t)(3 * nf + 1));
    int64_t nc = select_edges(m, cand);
    int64_t demoted = 0;
    if (mlp) {
        /* score every candidate first, then set the low ones aside */
        uint8_t *low = xalloc((size_t)nc + 1);
        float x[NFEAT];
        for (int64_t c = 0; c < nc; c++) {
            edge_features(m, ovl, cand[c], x);
            low[c] = mlp_logit(mlp, x) < (double)mlp->threshold;
        }
        for (int64_t c = 0; c < nc; c++)
            if (low[c]) { m->key[cand[c]] = KEY_MAX; demoted++; }
        free(low);
        if (demoted) nc = select_edges(m, cand);
    }
    uint8_t *reason = xalloc((size_t)nc + 1);
    double *vbar = xalloc(sizeof(double) * 3 * (size_t)(nc + 1));

    /* R7 */
    int64_t npass = 0;
    for (int64_t c = 0; c < nc; c++) {
        int64_t h = cand[c];
        int32_t a = m->F[h], b = m->F[3 * (h / 3) + (h % 3 + 1) % 3];
        double cost = edge_cost(m, a, b, opt->w_e, opt->w_s, vbar + 3 * c);
        (void)cost;
        reason[c] = (uint8_t)local_check(m, a, b, vbar + 3 * c);
        if (reason[c] == 0) npass++;
    }
    /* R8 */
    int64_t need = (count_alive_faces(m) - target_eff) / 2;
    int64_t nchosen = npass;
    if (npass > need) {
        int32_t *pass = xalloc(sizeof(int32_t) * (size_t)(npass + 1));
        uint64_t *pk = xalloc(sizeof(uint64_t) * (size_t)(nc + 1));
        int64_t k = 0;
        for (int64_t c = 0; c < nc; c++) {
            pk[c] = m->key[cand[c]];
            if (reason[c] == 0) pass[k++] = (int32_t)c;
        }
        g_sort_keys = pk;
        qsort(pass, (size_t)npass, sizeof(int32_t), cmp_by_key);
        for (int64_t i = need; i < npass; i++) reason[pass[i]] = 4;
        nchosen = need;
        free(pass);
        free(pk);
    }

    /* R9: apply every chosen collapse; remember the pre-round state */
    double *Vpre = xalloc(sizeof(double) * 3 * (size_t)nv);
    int32_t *Fpre = xalloc(sizeof(int32_t) * 3 * (size_t)nf);
    memcpy(Vpre, m->V, sizeof(double) * 3 * (size_t)nv);
    memcpy(Fpre, m->F, sizeof(int32_t) * 3 * (size_t)nf);
    int32_t *owner = xalloc(sizeof(int32_t) * (size_t)nf);
    for (int64_t f = 0; f < nf; f++) owner[f] = -1;
    uint8_t *applied = xalloc((size_t)nc + 1);
    int64_t *roff = xalloc(sizeof(int64_t) * (size_t)(nc + 1));
    int32_t *rfaces;
    {
        int64_t tot = 0;
        int32_t ring[RING_CAP];
        for (int64_t c = 0; c < nc; c++) {
            roff[c] = tot;
            if (reason[c] != 0) continue;
            int64_t h = cand[c];
            int32_t a = m->F[h], b = m->F[3 * (h / 3) + (h % 3 + 1) % 3];
            tot += ring_faces(m, a, b, ring, RING_CAP);
        }
        roff[nc] = tot;
        rfaces = xalloc(sizeof(int32_t) * (size_t)(tot + 1));
        for (int64_t c = 0; c < nc; c++) {
            if (reason[c] != 0) continue;
            int64_t h = cand[c];
            int32_t a = m->F[h], b = m->F[3 * (h / 3) + (h % 3 + 1) % 3];
            ring_faces(m, a, b, rfaces + roff[c], RING_CAP);
        }
    }
    int64_t changed = 0;
    for (int64_t c = 0; c < nc; c++) {
        if (reason[c] != 0) continue;
        applied[c] = 1;
        int64_t h = cand[c];
        int32_t a = m->F[h], b = m->F[3 * (h / 3) + (h % 3 + 1) % 3];
        int32_t s = a < b ? a : b, r = a < b ? b : a;
        for (int64_t i = roff[c]; i < roff[c + 1]; i++) {
            int32_t f = rfaces[i];
            if (owner[f] >= 0) { fprintf(stderr, "oracle: regions overlap\n"); abort(); }
            owner[f] = (int32_t)c;
            if (face_has(m, f, s) && face_has(m, f, r)) {
                m->falive[f] = 0;
            } else {
                changed++;
                for (int k = 0; k < 3; k++)
                    if (m->F[3 * (int64_t)f + k] == r) m->F[3 * (int64_t)f + k] = s;
            }
        }
        m->V[3 * (int64_t)s + 0] = vbar[3 * c + 0];
        m->V[3 * (int64_t)s + 1] = vbar[3 * c + 1];
        m->V[3 * (int64_t)s + 2] = vbar[3 * c + 2];
    }

    /* R11: check / undo until no changed triangle intersects anything */
    int64_t iters = 0;
    uint8_t *mark = xalloc((size_t)nc + 1);
    int64_t *stamp = xalloc(sizeof(int64_t) * (size_t)nf);
    for (int64_t f = 0; f < nf; f++) stamp[f] = -1;
    int64_t stamp_id = 0;
    int32_t *ovl_new = ovl ? xalloc(sizeof(int32_t) * (size_t)nf) : NULL;
    for (;;) {
        ogrid G;
        grid_build(m, &G);
        if (ovl_new && iters == 0) {
            /* overlap counts of the changed faces on the tentative mesh */
            for (int64_t t = 0; t < nf; t++) {
                if (!m->falive[t] || owner[t] < 0 || !applied[owner[t]]) continue;
                ovl_new[t] = overlap_count(m, &G, t, stamp, stamp_id++);
            }
        }
        memset(mark, 0, (size_t)nc + 1);
        undo_ctx uc = {m, owner, applied, mark, 0};
        for (int64_t t = 0; t < nf; t++) {
            if (!m->falive[t] || owner[t] < 0 || !applied[owner[t]]) continue;
            query_face(m, &G, t, stamp, stamp_id++, mark_owners, &uc);
        }
        grid_free(&G);
        if (uc.nmark == 0) break;
        iters++;
        for (int64_t c = 0; c < nc; c++) {
            if (!mark[c]) continue;
            applied[c] = 0;
            reason[c] = 3;
            int64_t h = cand[c];
            int32_t a = Fpre[h], b = Fpre[3 * (h / 3) + (h % 3 + 1) % 3];
            int32_t s = a < b ? a : b;
            for (int k = 0; k < 3; k++) m->V[3 * (int64_t)s + k] = Vpre[3 * (int64_t)s + k];
            for (int64_t i = roff[c]; i < roff[c + 1]; i++) {
                int32_t f = rfaces[i];
                for (int k = 0; k < 3; k++) m->F[3 * (int64_t)f + k] = Fpre[3 * (int64_t)f + k];
                m->falive[f] = 1;
            }
        }
    }
    free(mark);
    free(stamp);

    /* R12: commit */
    int64_t commits = 0;
    for (int64_t c = 0; c < nc; c++) {
        if (!applied[c]) continue;
        commits++;
        int64_t h = cand[c];
        int32_t a = Fpre[h], b = Fpre[3 * (h / 3) + (h % 3 + 1) % 3];
        m->valive[a < b ? b : a] = 0;
    }
    if (ovl_new) {
        for (int64_t t = 0; t < nf; t++)
            if (m->falive[t] && owner[t] >= 0 && applied[owner[t]]) ovl[t] = ovl_new[t];
        free(ovl_new);
    }
    out->demoted = demoted;
    out->retry = mlp && demoted > 0 && commits == 0;
    if (!stop_after_check && !out->retry) {
        uint8_t *nflags = xalloc((size_t)(3 * nf));
        for (int64_t c = 0; c < nc; c++) {
            if (reason[c] >= 1 && reason[c] <= 3) {
                nflags[cand[c]] = 1;
                nflags[m->twin[cand[c]]] = 1;
            }
        }
        if (commits == 0)
            for (int64_t h = 0; h < 3 * nf; h++) nflags[h] |= m->flags[h];
        free(m->flags);
        m->flags = nflags;
        m->streak = commits == 0 ? m->streak + 1 : 0;
    }

    out->ncand = nc;
    out->cand = cand;
    out->reason = reason;
    out->vbar = vbar;
    out->passing = npass;
    out->chosen = nchosen;
    out->changed = changed;
    out->undo_iters = iters;
    out->commits = commits;
    free(Vpre); free(Fpre); free(owner); free(applied); free(roff); free(rfaces);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* exported entry points (ctypes)                                            */
/* ------------------------------------------------------------------------ */

static void mesh_init(omesh *m, const double *V, int64_t nv, const int32_t *F, int64_t nf) {
    memset(m, 0, sizeof(*m));
    m->nv = nv;
    m->nf = nf;
    m->V = xalloc(sizeof(double) * 3 * (size_t)nv);
    m->F = xalloc(sizeof(int32_t) * 3 * (size_t)nf);
    memcpy(m->V, V, sizeof(double) * 3 * (size_t)nv);
    memcpy(m->F, F, sizeof(int32_t) * 3 * (size_t)nf);
    m->falive = xalloc((size_t)nf);
    m->valive = xalloc((size_t)nv);
    m->flags = xalloc((size_t)(3 * nf));
    memset(m->falive, 1, (size_t)nf);
    memset(m->valive, 1, (size_t)nv);
}

static void mesh_free(omesh *m) {
    free(m->V); free(m->F); free(m->falive); free(m->valive); free(m->flags);
    free(m->inc_off); free(m->inc); free(m->twin); free(m->Q); free(m->key);
}

static int check_input(const int32_t *F, int64_t nf, int64_t nv) {
    if (nv <= 0 || nf <= 0 || nf > (INT32_MAX / 3)) return -1;
    for (int64_t i = 0; i < 3 * nf; i++)
        if (F[i] < 0 || F[i] >= nv) return -1;
    return 0;
}

int oracle_quadrics(const double *V, int64_t nv, const int32_t *F, int64_t nf, double *Q) {
    if (check_input(F, nf, nv)) return -1;
    omesh m;
    mesh_init(&m, V, nv, F, nf);
    compute_quadrics(&m);
    memcpy(Q, m.Q, sizeof(double) * 10 * (size_t)nv);
    mesh_free(&m);
    return 0;
}

int oracle_keys(const double *V, int64_t nv, const int32_t *F, int64_t nf, const uint8_t *flags,
                double w_e, double w_s, uint64_t *keys) {
    if (check_input(F, nf, nv)) return -1;
    omesh m;
    mesh_init(&m, V, nv, F, nf);
    if (flags) memcpy(m.flags, flags, (size_t)(3 * nf));
    int err = build_adjacency(&m);
    if (!err) {
        compute_quadrics(&m);
        compute_keys(&m, w_e, w_s);
        memcpy(keys, m.key, sizeof(uint64_t) * (size_t)(3 * nf));
    }
    mesh_free(&m);
    return err;
}

int oracle_select(const double *V, int64_t nv, const int32_t *F, int64_t nf, const uint8_t *flags,
                  double w_e, double w_s, int32_t *cand, int64_t *ncand) {
    if (check_input(F, nf, nv)) return -1;
    omesh m;
    mesh_init(&m, V, nv, F, nf);
    if (flags) memcpy(m.flags, flags, (size_t)(3 * nf));
    int err = build_adjacency(&m);
    if (!err) {
        compute_quadrics(&m);
        compute_keys(&m, w_e, w_s);
        *ncand = select_edges(&m, cand);
    }
    mesh_free(&m);
    return err;
}

/* one round up to the end of the check/undo loop: the candidates, their
 * placements and their outcome (0 kept, 1 link, 2 flip/degenerate,
 * 3 intersection, 4 capped by the face target) */
int oracle_check(const double *V, int64_t nv, const int32_t *F, int64_t nf, const uint8_t *flags,
                 double w_e, double w_s, int64_t target, int32_t prefilter, int32_t key_mode, int32_t *cand,
                 int64_t *ncand,
                 double *vbar, uint8_t *reason, int64_t *undo_iters) {
    if (check_input(F, nf, nv)) return -1;
    omesh m;
    mesh_init(&m, V, nv, F, nf);
    if (flags) memcpy(m.flags, flags, (size_t)(3 * nf));
    oracle_opts o = {w_e, w_s, 4, -1, 0.0, prefilter, key_mode};
    round_out r;
    int err = run_round(&m, target - (target % 2), &o, &r, 1, NULL, NULL);
    if (!err) {
        *ncand = r.ncand;
        memcpy(cand, r.cand, sizeof(int32_t) * (size_t)r.ncand);
        memcpy(vbar, r.vbar, sizeof(double) * 3 * (size_t)r.ncand);
        memcpy(reason, r.reason, (size_t)r.ncand);
        if (undo_iters) *undo_iters = r.undo_iters;
        free(r.cand); free(r.reason); free(r.vbar);
    }
    mesh_free(&m);
    return err;
}

/* training rows of the learned proposal: the features of each round's
 * candidates and whether the candidate was committed (1) or rejected by a
 * check (0); candidates left out by the face target give no row */
typedef struct {
    float *X;
    uint8_t *y;
    int64_t cap, n;
} collect_buf;

static int run_impl(const double *V, int64_t nv, const int32_t *F, int64_t nf,
                    const uint8_t *flags_in, int32_t streak_in, int64_t target, const oracle_opts *opt,
                    double *Vout, int64_t *nv_out, int32_t *Fout, int64_t *nf_out,
                    uint8_t *flags_out, int32_t *streak_out, oracle_stats *st,
                    oracle_round_log *log, int64_t log_cap, const oracle_mlp *mlp, collect_buf *col,
                    int64_t *learned_info) {
    if (check_input(F, nf, nv) || target < 0) return -1;
    omesh m;
    mesh_init(&m, V, nv, F, nf);
    if (flags_in) memcpy(m.flags, flags_in, (size_t)(3 * nf));
    m.streak = streak_in;
    memset(st, 0, sizeof(*st));
    int32_t *ovl = NULL;
    if (mlp || col) {
        ovl = xalloc(sizeof(int32_t) * (size_t)nf);
        overlap_init(&m, ovl);
    }
    int64_t teff = target - (target % 2);
    int err = 0;
    int prev_rejected = 0; /* the network is consulted only after a round whose checks rejected something */
    for (;;) {
        int64_t falive = count_alive_faces(&m);
        if (falive <= teff) { st->status = 0; break; }
        if (m.streak >= opt->tolerance) { st->status = 1; break; }
        if (opt->max_rounds >= 0 && st->rounds >= opt->max_rounds) { st->status = 2; break; }
        int64_t valive = 0;
        for (int64_t v = 0; v < m.nv; v++) valive += m.valive[v];
        round_out r;
        float *feat = NULL;
        if (col) {
            /* features of this round's candidates, taken before the round
             * changes the mesh (the plain selection; col and mlp exclude
             * each other) */
            err = build_adjacency(&m);
            if (err) break;
            compute_quadrics(&m);
            compute_keys_capped(&m, opt->w_e, opt->w_s, opt->cost_target, opt->key_mode);
            int32_t *c0 = xalloc(sizeof(int32_t) * (size_t)(3 * m.nf + 1));
            int64_t n0 = select_edges(&m, c0);
            feat = xalloc(sizeof(float) * NFEAT * (size_t)(n0 + 1));
            for (int64_t c = 0; c < n0; c++) edge_features(&m, ovl, c0[c], feat + NFEAT * c);
            free(c0);
        }
        err = run_round(&m, teff, opt, &r, 0, prev_rejected ? mlp : NULL, ovl);
        if (err) { free(feat); break; }
        if (learned_info) learned_info[0] += r.demoted;
        if (r.retry) {
            /* nothing committed with candidates set aside: the plain round */
            free(r.cand); free(r.reason); free(r.vbar);
            if (learned_info) learned_info[1]++;
            err = run_round(&m, teff, opt, &r, 0, NULL, ovl);
            if (err) break;
        }
        if (col) {
            for (int64_t c = 0; c < r.ncand && col->n < col->cap; c++) {
                if (r.reason[c] > 3) continue;
                memcpy(col->X + NFEAT * col->n, feat + NFEAT * c, sizeof(float) * NFEAT);
                col->y[col->n] = r.reason[c] == 0;
                col->n++;
            }
            free(feat);
        }
        int64_t rl = 0, rf = 0, ri = 0, cp = 0;
        for (int64_t c = 0; c < r.ncand; c++) {
            rl += r.reason[c] == 1;
            rf += r.reason[c] == 2;
            ri += r.reason[c] == 3;
            cp += r.reason[c] == 4;
        }
        prev_rejected = rl + rf + ri > 0;
        if (log && st->rounds < log_cap) {
            oracle_round_log *L = log + st->rounds;
            L->faces = falive; L->verts = valive; L->edges = falive * 3 / 2;
            L->candidates = r.ncand; L->passing = r.passing; L->chosen = r.chosen;
            L->changed_faces = r.changed; L->undo_iters = r.undo_iters; L->commits = r.commits;
            L->rej_link = rl; L->rej_flip = rf; L->rej_isect = ri; L->capped = cp;
        }
        st->rounds++;
        st->commits += r.commits;
        st->candidates += r.ncand;
        st->rej_link += rl; st->rej_flip += rf; st->rej_isect += ri; st->capped += cp;
        st->undo_hist[r.undo_iters < 4 ? r.undo_iters : 4]++;
        const int64_t selected = r.ncand;
        free(r.cand); free(r.reason); free(r.vbar);
        /* with a cost target, a round that selects nothing ends the run: every
         * edge is then flagged or costs more than the target, and the next
         * round would be the same */
        if (opt->cost_target > 0 && selected == 0) { st->status = 0; break; }
    }
    if (!err) {
        int32_t *vmap = xalloc(sizeof(int32_t) * (size_t)m.nv);
        int64_t k = 0;
        for (int64_t v = 0; v < m.nv; v++) {
            vmap[v] = -1;
            if (!m.valive[v]) continue;
            vmap[v] = (int32_t)k;
            memcpy(Vout + 3 * k, m.V + 3 * v, sizeof(double) * 3);
            k++;
        }
        *nv_out = k;
        int64_t j = 0;
        for (int64_t f = 0; f < m.nf; f++) {
            if (!m.falive[f]) continue;
            for (int c = 0; c < 3; c++) {
                Fout[3 * j + c] = vmap[m.F[3 * f + c]];
                if (flags_out) flags_out[3 * j + c] = m.flags[3 * f + c];
            }
            j++;
        }
        *nf_out = j;
        if (streak_out) *streak_out = m.streak;
        free(vmap);
    }
    free(ovl);
    mesh_free(&m);
    return err;
}

/* The whole method: rounds until the face target, the tolerance or
 * max_rounds.  Output is the stable compaction of alive vertices and faces;
 * flags_out (3 * nf_out, may be NULL) are the invalid-edge flags in the output
 * numbering. */
int oracle_run(const double *V, int64_t nv, const int32_t *F, int64_t nf,
               const uint8_t *flags_in, int32_t streak_in, int64_t target, const oracle_opts *opt,
               double *Vout, int64_t *nv_out, int32_t *Fout, int64_t *nf_out,
               uint8_t *flags_out, int32_t *streak_out, oracle_stats *st,
               oracle_round_log *log, int64_t log_cap) {
    return run_impl(V, nv, F, nf, flags_in, streak_in, target, opt, Vout, nv_out, Fout, nf_out, flags_out,
                    streak_out, st, log, log_cap, NULL, NULL, NULL);
}

/* The method with the learned proposal (mlp); learned_info (2 entries, may
 * be NULL) gets the candidates set aside and the rounds run again plain. */
int oracle_run_learned(const double *V, int64_t nv, const int32_t *F, int64_t nf, int64_t target,
                       const oracle_opts *opt, const oracle_mlp *mlp, double *Vout, int64_t *nv_out,
                       int32_t *Fout, int64_t *nf_out, oracle_stats *st, int64_t *learned_info) {
    if (learned_info) learned_info[0] = learned_info[1] = 0;
    if (opt->key_mode) return -1; /* the features read the float32 cost from the key */
    return run_impl(V, nv, F, nf, NULL, 0, target, opt, Vout, nv_out, Fout, nf_out, NULL, NULL, st, NULL, 0,
                    mlp, NULL, learned_info);
}

/* The plain method, logging training rows (X: cap x 32 floats, y: cap). */
int oracle_collect(const double *V, int64_t nv, const int32_t *F, int64_t nf, int64_t target,
                   const oracle_opts *opt, float *X, uint8_t *y, int64_t cap, int64_t *n,
                   double *Vout, int64_t *nv_out, int32_t *Fout, int64_t *nf_out, oracle_stats *st) {
    /* logged rows come from the plain selection with R4's keys */
    if (opt->key_mode || opt->prefilter) return -1;
    collect_buf col = {X, y, cap, 0};
    int err = run_impl(V, nv, F, nf, NULL, 0, target, opt, Vout, nv_out, Fout, nf_out, NULL, NULL, st, NULL, 0,
                       NULL, &col, NULL);
    *n = col.n;
    return err;
}

/* features of the given edges (half-edge ids) of a mesh, with the overlap
 * counts of the mesh itself (as at the start of a run) */
int oracle_features(const double *V, int64_t nv, const int32_t *F, int64_t nf, const int32_t *edges,
                    int64_t ne, double w_e, double w_s, float *X, int32_t *ovl_out) {
    if (check_input(F, nf, nv)) return -1;
    omesh m;
    mesh_init(&m, V, nv, F, nf);
    int err = build_adjacency(&m);
    if (!err) {
        compute_quadrics(&m);
        compute_keys(&m, w_e, w_s);
        int32_t *ovl = xalloc(sizeof(int32_t) * (size_t)nf);
        overlap_init(&m, ovl);
        for (int64_t i = 0; i < ne; i++) edge_features(&m, ovl, edges[i], X + NFEAT * i);
        if (ovl_out) memcpy(ovl_out, ovl, sizeof(int32_t) * (size_t)nf);
        free(ovl);
    }
    mesh_free(&m);
    return err;
}

/* the network's logit for each of n quantised feature rows */
int oracle_mlp_logits(const oracle_mlp *M, const float *X, int64_t n, double *out) {
    for (int64_t i = 0; i < n; i++) out[i] = mlp_logit(M, X + NFEAT * i);
    return 0;
}

int64_t oracle_sizeof_mlp(void) { return (int64_t)sizeof(oracle_mlp); }

int oracle_tri_pair(const double *P9, const int32_t *ip, const double *Q9, const int32_t *iq) {
    const double *P[3] = {P9, P9 + 3, P9 + 6};
    const double *Q[3] = {Q9, Q9 + 3, Q9 + 6};
    return o_tri_pair(P, ip, Q, iq);
}

int oracle_degenerate(const double *P9) { return o_degenerate(P9, P9 + 3, P9 + 6); }

typedef struct {
    int32_t *pairs;
    int64_t cap, n;
} pair_list;

static void add_pair(void *vctx, int64_t t, int64_t u) {
    pair_list *p = vctx;
    if (t > u) return; /* each unordered pair once */
    if (p->n < p->cap) {
        p->pairs[2 * p->n] = (int32_t)t;
        p->pairs[2 * p->n + 1] = (int32_t)u;
    }
    p->n++;
}

/* whole-mesh self-intersection pairs (t < u), in ascending (t, u) order */
int oracle_self_intersections(const double *V, int64_t nv, const int32_t *F, int64_t nf,
                              int32_t *pairs, int64_t cap, int64_t *npairs) {
    if (check_input(F, nf, nv)) return -1;
    omesh m;
    mesh_init(&m, V, nv, F, nf);
    ogrid G;
    grid_build(&m, &G);
    int64_t *stamp = xalloc(sizeof(int64_t) * (size_t)nf);
    for (int64_t f = 0; f < nf; f++) stamp[f] = -1;
    pair_list pl = {pairs, cap, 0};
    for (int64_t t = 0; t < nf; t++) query_face(&m, &G, t, stamp, t, add_pair, &pl);
    *npairs = pl.n;
    free(stamp);
    grid_free(&G);
    mesh_free(&m);
    return 0;
}

/* input precondition: closed edge-manifold (every half-edge has exactly one
 * opposite), vertex-manifold (each vertex star is one fan), no exactly
 * degenerate face.  0 ok, -2 not manifold, -4 degenerate face. */
int oracle_validate(const double *V, int64_t nv, const int32_t *F, int64_t nf) {
    if (check_input(F, nf, nv)) return -1;
    omesh m;
    mesh_init(&m, V, nv, F, nf);
    int err = build_adjacency(&m);
    if (!err) {
        for (int64_t f = 0; f < nf && !err; f++) {
            const int32_t *t = F + 3 * f;
            if (t[0] == t[1] || t[1] == t[2] || t[0] == t[2]) err = -2;
            else if (o_degenerate(V + 3 * (int64_t)t[0], V + 3 * (int64_t)t[1], V + 3 * (int64_t)t[2])) err = -4;
        }
        /* each vertex: walking around it from one face must visit all its faces */
        for (int64_t v = 0; v < nv && !err; v++) {
            int64_t deg = m.inc_off[v + 1] - m.inc_off[v];
            if (deg == 0) continue;
            int32_t f0 = m.inc[m.inc_off[v]];
            int c0 = 0;
            while (F[3 * (int64_t)f0 + c0] != v) c0++;
            int64_t h0 = 3 * (int64_t)f0 + c0, h = h0, cnt = 0;
            do {
                int64_t prev = 3 * (h / 3) + (h % 3 + 2) % 3; /* incoming to v */
                h = m.twin[prev];                              /* outgoing from v */
                cnt++;
            } while (h != h0 && cnt <= deg);
            if (cnt != deg) err = -2;
        }
    }
    mesh_free(&m);
    return err;
}

/* sizes of the oracle's public structs, for binding checks */
int64_t oracle_sizeof_opts(void) { return (int64_t)sizeof(oracle_opts); }
int64_t oracle_sizeof_stats(void) { return (int64_t)sizeof(oracle_stats); }
int64_t oracle_sizeof_round_log(void) { return (int64_t)sizeof(oracle_round_log); }

/* leaf functions exported for the closed-form pins */
double oracle_skinny(const double *P9) { return skinny_term(P9, P9 + 3, P9 + 6); }

uint64_t oracle_make_key(double cost, uint32_t edge_id) { return make_key(cost, edge_id); }

double oracle_quadric_eval(const double *q10, const double *v) { return quadric_eval(q10, v); }

/* cost and placement of collapsing edge (a, b) of a closed mesh */
int oracle_edge_cost(const double *V, int64_t nv, const int32_t *F, int64_t nf, int32_t a, int32_t b,
                     double w_e, double w_s, double *cost, double *vbar) {
    if (check_input(F, nf, nv)) return -1;
    omesh m;
    mesh_init(&m, V, nv, F, nf);
    int err = build_adjacency(&m);
    if (!err) {
        compute_quadrics(&m);
        *cost = edge_cost(&m, a, b, w_e, w_s, vbar);
    }
    mesh_free(&m);
    return err;
}
